// Internal host-side structures of the tmcs library.
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "tmcs.h"

namespace tmcs {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
tmcs_status fail(tmcs_status st, const std::string& msg);

// ----------------------------------------------------------------- GF(2)
// Dense bit rows: vector of uint64 words, bit j of row = word j/64, bit j%64.
using BitRow = std::vector<uint64_t>;
int gf2_rank_rows(std::vector<BitRow> rows, int ncols);

// ----------------------------------------------------------------- codes
struct CodeBlock {
  int kind = TMCS_SC;
  int n = 0, k = 0;
  int nx = 0, nz = 0;                     // X / Z checks
  std::vector<std::vector<int>> hx, hz;   // check -> data qubits (ascending)
  std::vector<std::vector<int>> lz;       // logical Z supports
  // schedule: per CX layer, (check, data) pairs for X and Z checks
  int layers = 0;
  std::vector<std::vector<std::pair<int, int>>> xs, zs;
};
tmcs_status make_code(const tmcs_circuit_spec& s, CodeBlock* out);

// --------------------------------------------------------------- circuits
enum OpKind : uint8_t {
  OP_R, OP_RX, OP_M, OP_MX, OP_H, OP_CX, OP_BELL, OP_CXREC, OP_CZREC,
  OP_XERR, OP_ZERR, OP_DEP1, OP_DEP2, OP_TICK, OP_DET, OP_OBS
};
struct Op {
  OpKind kind;
  double p = 0.0;              // noise ops
  int obs = 0;                 // OP_OBS index
  std::vector<int32_t> t;      // qubits / pairs / (rec, q) pairs / records
};

struct Circuit {
  tmcs_circuit_spec spec{};
  CodeBlock code;
  std::vector<Op> ops;
  int num_qubits = 0, num_meas = 0, num_dets = 0, num_obs = 0;
  int64_t num_sites = 0;
  int64_t final_meas = 0;
  void* device = nullptr;      // device-side program and scratch (sample.hip)
};

tmcs_status build_circuit(const tmcs_circuit_spec& s, Circuit* c);
std::string circuit_text(const Circuit& c);
void circuit_counts(const Circuit& c, int64_t info[TMCS_INFO_LEN]);

// ------------------------------------------------------------------- DEM
constexpr int MAX_OBS = 256;                  // logical observables a circuit may have

struct Dem {
  int rows = 0, cols = 0, nobs = 0;
  int64_t edges = 0;
  int rank = 0;
  int64_t undetectable = 0;
  std::vector<int32_t> col_ptr, row_idx;      // CSC, rows ascending
  std::vector<int32_t> row_ptr, col_idx;      // CSR, cols ascending
  std::vector<int32_t> csc_edge;              // CSC position -> CSR edge id
  std::vector<double> priors;
  int obs_words = 1;                          // ceil(nobs / 64), at least 1
  std::vector<uint64_t> obs_mask;             // [cols][obs_words]: bit o of word o/64 = flips observable o
  int max_row_deg = 0, max_col_deg = 0;
  void* device = nullptr;                     // decoder-side device copy (decode.hip)
};
tmcs_status build_dem(const Circuit& c, Dem* d);
tmcs_status dem_distance(const Dem& D, int max_active, int max_weight, int64_t max_states, int32_t* weight);

// Probability of one independent mechanism of a channel (shared by the DEM
// builder; definitions in dem.cpp).
double mechanism_prob(OpKind k, double p);
int channel_components(OpKind k);

}  // namespace tmcs

struct tmcs_circuit { tmcs::Circuit c; };
struct tmcs_dem { tmcs::Dem d; };
