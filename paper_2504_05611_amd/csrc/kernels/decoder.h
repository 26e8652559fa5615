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
// the smaller first windows (their shots that need more rows go to the full one)
constexpr int WIN_SMALL_MW = 8;
constexpr int WIN_SMALL_ROWS = 64 * WIN_SMALL_MW;
constexpr int WIN_MID_MW = 16;
constexpr int WIN_MID_ROWS = 64 * WIN_MID_MW;
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

// Loads and stores through the global address space.  A pointer the kernel
// reads from memory (the per-item arguments of a multi launch) is generic to
// the compiler, which then emits flat accesses and waits for every
// outstanding memory operation before using any of them; these helpers keep
// such accesses global, so loads issued ahead stay in flight.
#define TMCS_GLOBAL_AS __attribute__((address_space(1)))
typedef int tmcs_v2i __attribute__((ext_vector_type(2)));
typedef int tmcs_v4i __attribute__((ext_vector_type(4)));
typedef float tmcs_v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int2 gload(const int2* p) {
  const tmcs_v2i v = *(const TMCS_GLOBAL_AS tmcs_v2i*)p;
  return make_int2(v.x, v.y);
}
__device__ __forceinline__ int4 gload(const int4* p) {
  const tmcs_v4i v = *(const TMCS_GLOBAL_AS tmcs_v4i*)p;
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float4 gload(const float4* p) {
  const tmcs_v4f v = *(const TMCS_GLOBAL_AS tmcs_v4f*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int32_t gload(const int32_t* p) { return *(const TMCS_GLOBAL_AS int32_t*)p; }
__device__ __forceinline__ float gload(const float* p) { return *(const TMCS_GLOBAL_AS float*)p; }
__device__ __forceinline__ uint64_t gload(const uint64_t* p) { return *(const TMCS_GLOBAL_AS uint64_t*)p; }
__device__ __forceinline__ void gstore(float4* p, const float4 x) {
  tmcs_v4f v;
  v.x = x.x; v.y = x.y; v.z = x.z; v.w = x.w;
  *(TMCS_GLOBAL_AS tmcs_v4f*)p = v;
}
__device__ __forceinline__ void gstore(float* p, const float x) { *(TMCS_GLOBAL_AS float*)p = x; }

// A copy of a workgroup-uniform struct read from device memory, every word
// passed through readfirstlane, so that the compiler keeps the fields in
// scalar registers (a plain copy lands in vector registers, one per word:
// the memory might be written by the kernel, so no scalar load is used).
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized struct");
  T out;
  const uint32_t* src = (const uint32_t*)p;
  uint32_t* dst = (uint32_t*)&out;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return out;
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

// ------------------------------------------------------------------ BP
// Schedule records of the BP passes (int4 = {x, y, z, w}).
//   check pass: x = v | flags, y = CSR edge e, z = check c (edges of a check are
//               consecutive in one lane, in CSR order)
//   var pass:   x = v | flags, y = CSR edge e, z = check c, w = lambda_v bits
//               (entries of a column are consecutive in one lane, in CSC order)
//   both:       bits R_SH.. of x = 2 + the edge's position within its check
//               (0 where the check has more than PK_MAX_DEG edges)
// The packed-state team kernel (PK) reads one int32 per edge and pass instead:
//   check pass: v' | position bits | flags;  var pass: c' | position bits | flags
// over checks and columns grouped by degree into chunks of 64 (one per lane of
// a wave, padded with no-op edges), so the flags are the same in every lane of
// a wave at every step; lane l's k-th check is at slot c' = k P + l and its
// k-th column at v' = k P + l.
// A team kernel gives every lane its own record list; the lanes kernel gives
// every wave one.
constexpr int32_t R_FIRST = 1 << 30;    // first edge of its check / column
constexpr int32_t R_LAST = (int32_t)(1u << 31);
constexpr int32_t R_SH = 25;
constexpr int32_t R_IDX = (1 << R_SH) - 1;
// Packed check state (team kernel, checks of at most PK_MAX_DEG edges): the
// last word of a check record holds s_c in bit 1 and, in bit 2 + j, the sign
// of the message to the check's j-th edge (s_c + sign parity + sgn q_e mod 2),
// so no per-edge sign byte is stored.
constexpr int PK_MAX_DEG = 30;

struct BPArgs {
  const int4* csched;        // [Kc][P] check-pass records
  const int4* vsched;        // [Kv][P] variable-pass records
  int32_t Kc, Kv;
  const int4* init;          // [m] check state of iteration 1 (n1, n2 bits, argmin edge, sign parity)
  const uint32_t* sign0;     // [E4 / 4] sign bytes of q at iteration 1
  const float* lam;
  const uint64_t* obs_mask;  // [ow][n]
  int32_t ow;
  int32_t m, n;
  int64_t E;
  int32_t E32;               // E as int32
  int32_t E4;                // E rounded up to a multiple of 4
  int32_t T;
  float alpha;
  const float* w;            // nullable [T][E]
  const uint64_t* synd;      // [chunk shots][mw] shot-major syndrome words
  int32_t mw;
  int64_t stride;            // words per row of pred
  int64_t shot0;             // first shot of this chunk (within the call)
  int64_t nshots;            // shots in this chunk
  const int32_t* queue;      // nullable: identity
  int32_t* counters;
  int32_t use_osd;
  int32_t* osd_queue;
  float* osd_llr;            // [chunk][n]
  uint64_t* pred;            // [k][stride]
  int32_t nobs;
  tmcs_decode_stats* stats;
  uint8_t* ehat;
  float* llr;
  int32_t* iters;
  uint8_t* flags;
  unsigned char* gstate;     // state in device memory: [grid][team_bytes]
  size_t team_bytes;
  const uint64_t* lone;      // nullable [mw]: checks without edges (such a check with s_c = 1 is never satisfied)
  uint64_t pm_lam[MAX_OW];   // observables flipped by the hard decision of lambda (a shot with s = 0)
  // single-pass kernel (bp_fused.hip)
  const int4* fsched;        // [Kf + 2][P][2] per-lane records, two int4 per edge
  int32_t Kf;
  const int32_t* csc_row;    // [E] check of each CSC entry (columns of degree >= 3)
  const int32_t* csc_edge;   // [E] CSR edge of each CSC entry
  uint64_t pm_iso[MAX_OW];   // observables of the columns without edges whose lambda < 0
  // packed-state team kernel.  State in device memory: 4-byte records over
  // degree chunks, lane l's k-th check at slot c' = k P + l and its k-th column
  // at v' = k P + l.  State in LDS: int2 records over longest-processing-time
  // lists, checks numbered in the order the lanes first reach them.
  const int2* pcs;           // LDS: [Kc + 2][P] check pass {v' | position | flags, c'}
  const int2* pvs;           // LDS: [Kv + 2][P] variable pass {c' | position | flags, lambda_v bits}
  const int32_t* pce;        // CSR edge of each check-pass record (per-edge weights), laid out as its records
  const int32_t* pve;        // the same for the variable pass
  const int32_t* vmap;       // [n] v -> v' (-1: a column without edges)
  const int32_t* corig;      // c' -> c; device memory: [Mpk + 2] (-1: an empty slot, the padding slot Mpk, the sink Mpk + 1)
  const int4* pinit;         // packed check state of iteration 1 by slot (s_c = 0; argmin as 2 + position)
  int32_t Mpk, Npk;          // check slots, column slots
  const int32_t* pcs4;       // [Kc4 + BP_AHEAD][P] check pass: v' | position | flags
  const int32_t* pvs4;       // [Kv4 + BP_AHEAD][P] variable pass: c' | position | flags
  const float* lamp;         // [Npk + 1] lambda_v by column slot
  int32_t Kc4, Kv4;          // Kc, Kv rounded up to BP_AHEAD (the arrays hold BP_AHEAD rows of padding past them)
};

// Steps whose loads the device-memory team kernel keeps in flight per lane.
constexpr int BP_AHEAD = 6;

// Several decode items' BP queues served by one launch.
struct BPMulti {
  const BPArgs* tab;         // device [n]: the items' arguments
  int32_t n;
  int32_t* next;             // device job counter shared by the launch (zeroed before it)
};
constexpr int MAX_MULTI = 16;

// BP with 64 shots per workgroup, one in each lane of every wave (bp_lanes.hip).
constexpr int LANES_WAVES = 16;         // waves per workgroup: each walks its own record list
constexpr int LANES_UNROLL = 8;         // records per batch of loads; lists are padded to a multiple
// Device-memory bytes of one lanes workgroup's state for an m x n DEM with E4 edge slots.
inline size_t lanes_slab_bytes(int m, int n, int E4) {
  const size_t b = (size_t)(m + 1) * 64 * 16 + (size_t)(n + 1) * 64 * 4 + ((size_t)E4 + 1) * 8;
  return (b + 255) & ~(size_t)255;
}
// mu.n > 0: a multi launch over mu's items (a is ignored); grid workgroups of LANES_WAVES waves.
tmcs_status launch_bp_lanes(const BPArgs& a, const BPMulti& mu, bool weighted, int grid, hipStream_t s);

// BP with one pass per iteration and its state in device memory (bp_fused.hip): a
// team of `threads` lanes per shot, as the two-pass team kernel.
// Device-memory bytes of one team's state: two buffers of check records, L, sign bytes.
inline size_t fused_team_bytes(int m, int n, int E4) {
  const size_t b = 2 * (size_t)(m + 1) * 16 + (size_t)n * 4 + (size_t)E4 + 4;
  return (b + 255) & ~(size_t)255;
}
tmcs_status launch_bp_fused(const BPArgs& a, const BPMulti& mu, bool weighted, int grid, int threads, hipStream_t s);

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
  int32_t* retry;            // PFX, and WIN's first window: jobs left open (counted in counters[4])
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
// mw: words of local rows, WIN_MW for the full window, WIN_SMALL_MW or WIN_MID_MW
// for a first window (a.retry receives what it leaves open).
tmcs_status launch_osd_win_multi(const OSDArgs& first, const OSDMulti& mu, int grid, size_t lds, hipStream_t s,
                                 int mw);
// Windowed OSD-0 (DEMs beyond the dense limits).
tmcs_status launch_osd_win(const OSDArgs& a, int grid, size_t lds, hipStream_t s, int mw);
// Dense OSD-0 on the npad - 1 smallest keys first (jobs the prefix does not settle go to a.retry).
tmcs_status dispatch_osd_pfx(int mw, bool bl, const OSDArgs& a, int grid, size_t lds, hipStream_t s);
// Dense OSD-0 (or OSD-CS) with a full sort of kpt keys per thread; bl: basis in LDS, one wave per shot.
tmcs_status dispatch_osd(int mw, int kpt, bool bl, const OSDArgs& a, int grid, size_t lds, hipStream_t s);
// Whether the one-wave variant with its basis in LDS applies (small DEMs).
bool osd_lds_basis_ok(int mw, int npad);

}  // namespace dec
}  // namespace tmcs
