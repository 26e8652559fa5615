// Device program of a circuit: the instruction stream the frame kernel runs.
#pragma once

#include <cstdint>
#include <vector>

#include "internal.h"

namespace tmcs {

// Layer kinds of the frame kernel.  Items of one layer touch disjoint frame
// words (except MEAS, which XORs into accumulator slots atomically), so a
// layer runs in parallel over (item, shot word) and layers are separated by a
// workgroup barrier.
enum LayerKind : int32_t {
  L_RESET = 0,   // item: q                      X = Z = 0
  L_H = 1,       // item: q                      swap X, Z
  L_CX = 2,      // item: c, t                   X[t] ^= X[c]; Z[c] ^= Z[t]
  L_MEAS = 3,    // item: q, basis, s0, s1       record (X or Z) XORed into slots mslot[s0..s1)
  L_FEED = 4,    // item: slot, q, pauli         X[q] (pauli 1) or Z[q] (pauli 3) ^= slot
  L_EMIT = 5,    // item: slot, out              det_out[out] = slot (out < 0: obs -out-1); slot = 0
  L_NOISE = 6,   // item: site, kind, q1, q2     apply the site's pre-generated events
  L_CLEAR = 7,   // item: slot                   slot = 0
};
inline int layer_item_width(int32_t kind) {
  switch (kind) {
    case L_RESET: case L_H: case L_CLEAR: return 1;
    case L_CX: case L_EMIT: return 2;
    case L_FEED: return 3;
    default: return 4;
  }
}

// Noise channel kinds on the device (site table)
enum NoiseKind : uint8_t { NK_XERR = 0, NK_ZERR = 1, NK_DEP1 = 2, NK_DEP2 = 3 };

struct Program {
  std::vector<int32_t> layers;  // 3 ints per layer: kind, count, data offset
  std::vector<int32_t> data;    // layer items
  std::vector<int32_t> mslots;  // slot lists of measurement items
  int nslots = 0;
  int num_layers = 0;
  // per noise site (circuit order): kind and index into the distinct-p table
  std::vector<uint8_t> site_kind;
  std::vector<uint16_t> site_tab;
  std::vector<double> tab_p;    // distinct event probabilities
  double events_per_shot = 0.0; // expected noise events per shot
};

tmcs_status compile_program(const Circuit& c, Program* p);

}  // namespace tmcs
