// Shared declarations of the decoder's translation units: the BP side
// (decode.hip: staging, BP, decode_run) and the OSD-0 side (osd.hip: the
// elimination kernels and their launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tmcs.h"

namespace tmcs {
namespace dec {

constexpr float BP_BIG = 1e30f;
constexpr int OSD_THREADS = 256;
constexpr int OSD_MAX_KEYS = 16384;
// windowed OSD-0: window length (sorted columns, power of two) and local rows
constexpr int WIN_KEYS = 2048;
constexpr int WIN_MW = 32;
constexpr int WIN_MAX_ROWS = 64 * WIN_MW;
// dense OSD-0 first tries this many smallest keys (one-wave and 256-thread variants)
constexpr int PFX_KEYS_WAVE = 128;
constexpr int PFX_KEYS_WG = 1024;
constexpr int32_t WIN_NONE = 0x7FFFFFFF;   // windowed OSD rowmap: row not touched by the window

// Observable masks: ow = ceil(nobs / 64) words per column, stored word-major
// ([ow][n]: word w of column v at w * n + v); at most MAX_OW words.
constexpr int MAX_OW = 4;

// Set the predicted flips of observables 64 word .. 64 word + 63 of one shot.
__device__ __forceinline__ void write_pred(uint64_t* pred, int64_t stride, int nobs, int64_t shot, uint64_t mask,
                                           int word) {
  for (int o = 0; o < 64 && 64 * word + o < nobs; ++o)
    if ((mask >> o) & 1ull)
      atomicOr((unsigned long long*)&pred[(int64_t)(64 * word + o) * stride + (shot >> 6)],
               (unsigned long long)(1ull << (shot & 63)));
}

__device__ __forceinline__ uint64_t block_xor_u64(uint64_t v, uint64_t* scratch) {
  if (threadIdx.x == 0) *scratch = 0ull;
  __syncthreads();
  if (v) atomicXor((unsigned long long*)scratch, (unsigned long long)v);
  __syncthreads();
  const uint64_t r = *scratch;
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ OSD-0
struct OSDArgs {
  const int32_t* col_ptr;
  const int32_t* csc_row;
  const uint64_t* obs_mask;  // [ow][n]
  int32_t ow;
  int32_t m, n, rank;
  const uint64_t* synd;      // [chunk shots][mw] shot-major syndrome words
  int32_t mw;
  int64_t stride;
  int64_t shot0;
  int32_t* counters;
  const int32_t* osd_queue;
  const float* osd_llr;
  uint64_t* basis;           // [grid][rank][W]
  uint64_t* pred;
  int32_t nobs;
  tmcs_decode_stats* stats;
  uint8_t* ehat;
  uint8_t* flags;
  int32_t npad;              // sort length (power of two >= n; WIN: window length)
  int32_t* rowmap;           // WIN: [grid][2][m] first window position touching a row, local row index
  int32_t win_rows;          // WIN: most local rows a window may hold (<= 64 * MW)
  const int32_t* jobs;       // nullable: job j is jobs[j] (a retry pass), else j
  int32_t cnt_total, cnt_next;   // counters[] holding the number of jobs and the next job
  int32_t* retry;            // PFX: jobs whose prefix did not span s (counted in counters[4])
  int32_t order;             // > 0: OSD-CS of this order (dense variants only)
};

// Several decode items' windowed OSD queues served by one launch (osd.hip).
constexpr int MAX_MULTI_OSD = 16;
struct OSDMulti {
  const OSDArgs* tab;        // device [n]: the items' arguments
  int32_t n;
  int32_t* next;             // device job counter shared by the launch (zeroed before it)
};

// OSD launchers (osd.hip).  grid workgroups, lds bytes of dynamic LDS.
// first: the first item's arguments (host copy; they fix the shared LDS layout).
tmcs_status launch_osd_win_multi(const OSDArgs& first, const OSDMulti& mu, int grid, size_t lds, hipStream_t s);
// Windowed OSD-0 (DEMs beyond the dense limits).
tmcs_status launch_osd_win(const OSDArgs& a, int grid, size_t lds, hipStream_t s);
// Dense OSD-0 on the npad - 1 smallest keys first (jobs the prefix does not settle go to a.retry).
tmcs_status dispatch_osd_pfx(int mw, bool bl, const OSDArgs& a, int grid, size_t lds, hipStream_t s);
// Dense OSD-0 (or OSD-CS) with a full sort of kpt keys per thread; bl: basis in LDS, one wave per shot.
tmcs_status dispatch_osd(int mw, int kpt, bool bl, const OSDArgs& a, int grid, size_t lds, hipStream_t s);
// Whether the one-wave variant with its basis in LDS applies (small DEMs).
bool osd_lds_basis_ok(int mw, int npad);

}  // namespace dec
}  // namespace tmcs
