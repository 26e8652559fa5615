// Batched BP + OSD-0 decoder and logical-error counting for gfx950.
//
// Min-sum belief propagation on the detector error model H (rows = detectors,
// columns = mechanisms), flooding schedule, prior LLRs lambda_v = ln((1-p)/p):
//   m_{c->v} = (-1)^{s_c} prod_{v' != v} sgn(q_{v'->c}) * (alpha * min_{v' != v} |q_{v'->c}|)
//   L_v = lambda_v + sum_{c ascending} m_{c->v};   q_{v->c} = L_v - m_{c->v}
//   stop when H [L < 0] = s (checked before every iteration and after the last)
// with sgn(0) = +1 and min over an empty set = 1e30.  alpha is a scalar, or
// w_t(c, v) per edge and iteration for weighted BP.  The paper names BP-OSD
// (Supplementary Note 7) without its equations; these are the standard ones.
//
// Layout: one workgroup decodes one shot at a time (persistent loop over a
// device queue).  Per-shot state lives in LDS in compressed form: L_v per
// column, (min1, min2, argmin edge, sign parity, syndrome bit) per check and one
// sign bit per edge; the messages m_{c->v} and q_{v->c} are recomputed from it,
// never stored.  Sums over a column run in ascending check order and no
// multiply-add is contracted, so results are bit-identical to an FP32 reference
// that follows the same order.
//
// OSD-0 (order 0 ordered-statistics decoding): columns sorted by (L_v, v)
// ascending (bitonic sort of 64-bit keys in LDS), the first rank(H) columns that
// are GF(2)-independent of the ones before them are kept, and H_S e_S = s is
// solved on them.  Elimination keeps an echelon basis of reduced columns in HBM
// (each vector = m syndrome bits followed by rank bits recording which kept
// columns it sums); candidates are reduced 256 at a time, one per thread, in
// registers, then among themselves in order.  DEMs beyond 2048 detectors or
// 16384 columns run the same elimination on a window of the sorted order (the
// smallest keys, found by radix selection, and the detectors they touch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../host/device.h"
#include "../host/timing.h"
#include "decoder.h"

namespace tmcs {

using namespace dec;

namespace {

struct DecodeDevice {
  int device = -1;
  int32_t *row_ptr = nullptr, *col_idx = nullptr, *col_ptr = nullptr, *csc_row = nullptr, *csc_edge = nullptr;
  float* lam = nullptr;
  uint64_t* obs_mask = nullptr;
  int4* init = nullptr;            // [m] BP check state of iteration 1
  uint32_t* sign0 = nullptr;       // [E4 / 4] sign bytes of iteration 1
  std::vector<int4> init_pk;       // host [m] packed check state of iteration 1 (empty: a check has > PK_MAX_DEG edges)
  int32_t E4 = 0;
  int32_t max_row_deg = 0;
  uint64_t* lone = nullptr;        // [mw] checks without edges (null: none)
  uint64_t pm_lam[MAX_OW] = {};    // observables of the hard decision of lambda
  uint64_t pm_iso[MAX_OW] = {};    // the same over the columns without edges
  // per-lane BP schedules, one per team size used so far
  struct Sched {
    int P = 0; int mode = 1; int Kc = 0, Kv = 0; int4* c = nullptr; int4* v = nullptr;
    int Kf = 0; int4* f = nullptr;   // single-pass records (built on first use)
    // packed-state team kernel (built on first use): 4-byte records over
    // degree chunks, check and column slots k P + l, lambda per column slot
    int32_t *pc4 = nullptr, *pv4 = nullptr, *corig4 = nullptr;
    int32_t *pce = nullptr, *pve = nullptr, *vmap = nullptr;
    int4* pinit4 = nullptr;
    float* lamp = nullptr;
    int32_t Mpk4 = 0, Npk = 0;
    int32_t Kc4 = 0, Kv4 = 0;        // list lengths rounded up to BP_AHEAD (arrays: [K4 + BP_AHEAD][P])
    // the LDS flavour (longest-processing-time lists of get_sched; checks numbered
    // in the order the lanes first reach them, columns i P + l; int2 records)
    int2 *pcL = nullptr, *pvL = nullptr;
    int32_t *pceL = nullptr, *pveL = nullptr, *vmapL = nullptr, *corigL = nullptr;
    int4* pinitL = nullptr;
    int32_t MpkL = 0, NpkL = 0;
  };
  std::vector<Sched> scheds;
  // scratch
  int32_t* counters = nullptr;     // [0] queue len, [1] bp next, [2] osd len, [3] osd next
  int32_t* queue = nullptr;
  int32_t* osd_queue = nullptr;
  float* osd_llr = nullptr;
  uint64_t* basis = nullptr;
  uint64_t* synd = nullptr;
  unsigned char* gstate = nullptr;  // BP state in device memory, one slab per team
  int32_t* rowmap = nullptr;        // windowed OSD: [grid][2][m] row tables (WIN_NONE between shots)
  int32_t* retry = nullptr;         // OSD jobs the sorted prefix did not settle
  size_t cap_queue = 0, cap_osd = 0, cap_llr = 0, cap_basis = 0, cap_synd = 0, cap_gstate = 0, cap_rowmap = 0;
  size_t cap_retry = 0;
};

__global__ void k_zero_words(uint64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_add_shots(tmcs_decode_stats* stats, unsigned long long n) {
  if (threadIdx.x == 0) atomicAdd((unsigned long long*)&stats->shots, n);
}

// Shots the compaction left out (all-zero syndrome) are converged: their
// all-zero hard decision satisfies s, as on the path that visits every shot.
__global__ void k_add_trivial(tmcs_decode_stats* stats, const int32_t* counters, unsigned long long n) {
  if (threadIdx.x != 0) return;
  const unsigned long long t = n - (unsigned long long)counters[0];
  atomicAdd((unsigned long long*)&stats->converged, t);
  atomicAdd((unsigned long long*)&stats->bp_iter_hist[0], t);
}

__global__ void k_zero_i32(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Detector-major bit planes -> shot-major syndrome words for the chunk
// [shot0, shot0 + nshots): one workgroup per 64-shot word and group of up to
// SYND_TILES 64-detector tiles, one 64 x 64 bit transpose through LDS per tile,
// so a shot's syndrome words are written together.  Workgroups go to the 8
// XCDs in turn, so the word index is remapped to give each XCD (and its L2) a
// contiguous range of words: a detector row's cache lines are then fetched by
// one L2, not eight.  gridDim.x is a multiple of 8, so every group of a word
// lands on the same XCD.
constexpr int N_XCD = 8;
constexpr int SYND_TILES = 8;
__global__ void __launch_bounds__(64) k_synd_transpose(const uint64_t* __restrict__ det, int32_t m, int64_t stride,
                                                       int64_t shot0, int64_t nshots, int32_t mw,
                                                       uint64_t* __restrict__ synd) {
  __shared__ uint64_t tile[64];
  const int lane = threadIdx.x;
  const int64_t per_xcd = gridDim.x / N_XCD;
  const int64_t w = (int64_t)(blockIdx.x % N_XCD) * per_xcd + blockIdx.x / N_XCD;   // shot word within the chunk
  if (w * 64 >= nshots) return;             // padding workgroup (uniform: before any barrier)
  const int64_t s = w * 64 + lane;
  const int rt1 = min(mw, (int)(blockIdx.y + 1) * SYND_TILES);
  for (int rt = blockIdx.y * SYND_TILES; rt < rt1; ++rt) {   // detector tiles of this group
    const int row = rt * 64 + lane;
    tile[lane] = row < m ? det[(int64_t)row * stride + (shot0 >> 6) + w] : 0ull;
    __syncthreads();
    uint64_t out = 0ull;
#pragma unroll 16
    for (int i = 0; i < 64; ++i) out |= ((tile[i] >> lane) & 1ull) << i;
    if (s < nshots) synd[s * mw + rt] = out;
    __syncthreads();                        // tile is refilled for the next detector tile
  }
}

// Queue the shots of the chunk whose syndrome is non-zero.  Same-address
// atomics serialise, so a workgroup (256 lanes) takes tiles of 16 x 256 shots
// and reserves the queue slots of a whole tile with one atomic.
constexpr int COMPACT_SLABS = 16;
__global__ void __launch_bounds__(256) k_compact(const uint64_t* __restrict__ synd, int32_t mw, int64_t nshots,
                                                 int32_t* __restrict__ queue, int32_t* __restrict__ counters) {
  __shared__ int s_wave[4];
  __shared__ int s_base;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  constexpr int64_t TILE = 256 * COMPACT_SLABS;
  for (int64_t t0 = (int64_t)blockIdx.x * TILE; t0 < nshots; t0 += (int64_t)gridDim.x * TILE) {
    uint64_t keep[COMPACT_SLABS];
    int tot = 0;
#pragma unroll
    for (int i = 0; i < COMPACT_SLABS; ++i) {
      const int64_t sh = t0 + i * 256 + threadIdx.x;
      uint64_t any = 0ull;
      if (sh < nshots)
        for (int k = 0; k < mw; ++k) any |= synd[sh * mw + k];
      keep[i] = __ballot(any != 0ull);
      tot += __popcll(keep[i]);
    }
    if (lane == 0) s_wave[wv] = tot;
    __syncthreads();
    if (threadIdx.x == 0) s_base = atomicAdd(&counters[0], s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3]);
    __syncthreads();
    int base = s_base;
    for (int w = 0; w < wv; ++w) base += s_wave[w];
#pragma unroll
    for (int i = 0; i < COMPACT_SLABS; ++i) {
      if ((keep[i] >> lane) & 1ull) queue[base + __popcll(keep[i] & below)] = (int32_t)(t0 + i * 256 + threadIdx.x);
      base += __popcll(keep[i]);
    }
    __syncthreads();   // s_wave and s_base are rewritten for the next tile
  }
}

// The same for wide syndromes (many detector words per shot, few shots per
// call, as in the large surface-code CNOTs): one wave per shot, its lanes
// reading the shot's words together, one queue slot per kept shot.  The queue
// order differs from k_compact's; every shot is decoded on its own, so nothing
// depends on it.
__global__ void __launch_bounds__(256) k_compact_wide(const uint64_t* __restrict__ synd, int32_t mw, int64_t nshots,
                                                      int32_t* __restrict__ queue, int32_t* __restrict__ counters) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t sh = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); sh < nshots; sh += waves) {
    uint64_t any = 0ull;
    for (int k = lane; k < mw; k += 64) any |= synd[sh * mw + k];
    if (__ballot(any != 0ull) && lane == 0) queue[atomicAdd(&counters[0], 1)] = (int32_t)sh;
  }
}

// BP over persistent teams: one workgroup (a "team" of P = blockDim.x lanes)
// decodes one shot at a time, with the whole per-shot state in LDS.  Work is
// split over the lanes by static schedules built once per DEM and team size
// (longest-processing-time assignment of whole checks, and of whole columns,
// to lanes), so every step of a pass is one edge per lane with no intra-pass
// synchronisation; a pass ends with one barrier.
//
// Per-shot LDS state (compressed): for every check (n1, n2) = the two smallest
// |q_{v->c}|, the argmin edge, the sign parity of the q's and the syndrome bit;
// one sign byte per edge (sign of q_{v->c}); L_v per column.  Messages are
// rebuilt from it: m_{c->v} = (-1)^{s_c + parity + sgn q_e} alpha_t(e) *
// (e == argmin ? n2 : n1).
//
// PK (every check of at most PK_MAX_DEG edges): no sign bytes.  A check
// record's last word holds s_c (bit 1) and the sign of the message to its j-th
// edge (bit 2 + j); the check pass collects the new signs in a register and
// writes them with the record, and both passes read a message's sign from the
// record they already load.  The argmin edge is kept as 2 + its position.
// Checks and columns are renumbered (c', v': the state and L slots in the
// order the lanes reach them) and the schedules hold 8-byte records, half the
// schedule bytes a team streams per iteration; the CSR edge of a record (for
// per-edge weights) comes from arrays of its own.  Results are the same.
//
// Iteration 1 needs no check pass: with q_{v->c} = lambda_v its state depends
// on the DEM alone (precomputed, plus the syndrome bit).  Iteration t is then a
// variable pass (L^t) followed by a check pass that tests H [L^t < 0] = s and,
// if t < T, builds the state of iteration t + 1.
// GSTATE: the per-shot state lives in this team's slab of device memory
// (a.gstate + blockIdx.x * a.team_bytes) instead of LDS, for DEMs whose state
// does not fit; the code is otherwise the same.
//
// MULTI: one launch decodes the queued shots of several decode items (a plan's
// instances, each with its own DEM, schedules, state and outputs): job g of a
// counter shared by the launch belongs to the item i with pref[i] <= g <
// pref[i + 1] (pref: prefix sums of the items' queue lengths), and the team
// switches to that item's arguments mu.tab[i].  Items are taken in order, so a
// team switches at most once per item; its statistics go to the item they
// belong to.  Weights are then per item (weights may be null: scalar alpha).

template <bool WEIGHTED, bool GSTATE, bool MULTI, bool PK>
__global__ void __launch_bounds__(1024) k_bp(BPArgs a, BPMulti mu) {
  extern __shared__ __align__(16) unsigned char sm[];
  unsigned char* base = nullptr;
  float4* state = nullptr;                            // [m + 1] (slot m: padding records); PK: [Mpk + 2] (LDS: [Mpk + 1])
  float* L = nullptr;                                 // [n]; PK: [Npk + 1] (slot Npk: +BIG for no-op edges)
  uint8_t* sgn = nullptr;                             // [E4 + 4] (byte E4: padding records); !PK only
  auto bind = [&]() {
    base = GSTATE ? a.gstate + (size_t)blockIdx.x * a.team_bytes : sm;
    state = (float4*)base;
    L = (float*)(state + (PK ? (GSTATE ? a.Mpk + 2 : a.Mpk + 1) : a.m + 1));
    sgn = (uint8_t*)(L + a.n);
  };
  // state and L accesses (device memory: kept global in a multi launch, whose slab pointer is read from memory)
  auto ld_state = [&](int c) -> float4 {
    if constexpr (GSTATE) return gload(state + c);
    else return state[c];
  };
  auto st_state = [&](int c, const float4 x) {
    if constexpr (GSTATE) gstore(state + c, x);
    else state[c] = x;
  };
  auto ld_L = [&](int v) -> float {
    if constexpr (GSTATE) return gload(L + v);
    else return L[v];
  };
  auto st_L = [&](int v, const float x) {
    if constexpr (GSTATE) gstore(L + v, x);
    else L[v] = x;
  };
  // schedule records and weights (a multi launch reads their pointers from memory)
  auto rec = [&](const auto* p) {
    if constexpr (MULTI) return gload(p);
    else return *p;
  };
  __shared__ int s_job, s_flag, s_pos, s_inst;
  __shared__ int s_unsat[2];
  __shared__ int s_pref[MAX_MULTI + 1];
  __shared__ unsigned long long s_pm[MAX_OW];
  __shared__ unsigned long long s_hist[TMCS_BP_HIST_BINS];   // written by thread 0 only
  const int tid = threadIdx.x, P = blockDim.x;
  int32_t total = 0;
  int cur = -1;                                       // MULTI: item the team works on
  if constexpr (!MULTI) {
    bind();
    total = a.queue ? a.counters[0] : (int32_t)a.nshots;
  } else if (tid == 0) {
    s_pref[0] = 0;
    for (int i = 0; i < mu.n; ++i)
      s_pref[i + 1] = s_pref[i] + (mu.tab[i].queue ? mu.tab[i].counters[0] : (int32_t)mu.tab[i].nshots);
  }
  unsigned long long c_nontriv = 0, c_conv = 0, c_osd = 0, c_iters = 0;   // thread 0
  for (int i = tid; i < TMCS_BP_HIST_BINS; i += P) s_hist[i] = 0ull;
  // statistics of the current item to its stats block, then reset
  auto flush = [&]() {
    __syncthreads();
    if (a.stats)
      for (int i = tid; i < TMCS_BP_HIST_BINS; i += P)
        if (s_hist[i]) atomicAdd((unsigned long long*)&a.stats->bp_iter_hist[i], s_hist[i]);
    if (tid == 0 && a.stats) {
      if (c_nontriv) atomicAdd((unsigned long long*)&a.stats->nontrivial, c_nontriv);
      if (c_conv) atomicAdd((unsigned long long*)&a.stats->converged, c_conv);
      if (c_osd) atomicAdd((unsigned long long*)&a.stats->osd, c_osd);
      if (c_iters) atomicAdd((unsigned long long*)&a.stats->bp_iters, c_iters);
    }
    c_nontriv = c_conv = c_osd = c_iters = 0;
    __syncthreads();
    for (int i = tid; i < TMCS_BP_HIST_BINS; i += P) s_hist[i] = 0ull;
    __syncthreads();
  };
  while (true) {
    if (tid == 0) {
      if constexpr (MULTI) {
        const int g = atomicAdd(mu.next, 1);
        int i = 0;
        while (i < mu.n && g >= s_pref[i + 1]) ++i;
        s_inst = i;
        s_job = i < mu.n ? g - s_pref[i] : 0;
      } else {
        s_job = atomicAdd(&a.counters[1], 1);
      }
      s_flag = 0;
      s_unsat[0] = 0;
      s_unsat[1] = 0;
      for (int w = 0; w < MAX_OW; ++w) s_pm[w] = 0ull;
    }
    __syncthreads();
    if constexpr (MULTI) {
      // (read through readfirstlane: the compiler then knows the value is uniform)
      const int inst = __builtin_amdgcn_readfirstlane(s_inst);
      if (inst != cur) {                              // uniform: the team moves to the next item
        if (cur >= 0) flush();
        if (inst >= mu.n) break;
        cur = inst;
        a = load_uniform(mu.tab + inst);
        bind();
      }
    }
    const int job = MULTI ? __builtin_amdgcn_readfirstlane(s_job) : s_job;
    if (!MULTI && job >= total) break;
    // per-item weights in a multi launch (null: scalar alpha)
    const bool use_w = WEIGHTED && (!MULTI || a.w != nullptr);
    const int64_t ls = a.queue ? a.queue[job] : job;
    const int64_t shot = a.shot0 + ls;
    // state of iteration 1, L = lambda, initial signs
    {
      const uint64_t* sy = a.synd + ls * a.mw;
      int fl = 0;
      if constexpr (PK) {
        // (L needs no start value: the variable pass writes every slot the check
        // pass reads, but slot Npk, which no-op check edges read)
        if (GSTATE && tid == 0) st_L(a.Npk, BP_BIG);
        for (int c = tid; c < (GSTATE ? a.Mpk + 2 : a.Mpk); c += P) {
          int4 s0 = gload(a.pinit + c);
          const int co = gload(a.corig + c);          // (-1: an empty, padding or sink slot)
          const int sb = co < 0 ? 0 : (int)((gload(sy + (co >> 6)) >> (co & 63)) & 1ull);
          fl |= sb;
          s0.w ^= sb ? (int)0xFFFFFFFEu : 0;   // s_c = 1 flips every message sign
          st_state(c, make_float4(__int_as_float(s0.x), __int_as_float(s0.y), __int_as_float(s0.z),
                                  __int_as_float(s0.w)));
        }
        // a detection event on a check without edges: never satisfied
        if (a.lone)
          for (int w = tid; w < a.mw; w += P)
            if (gload(sy + w) & gload(a.lone + w)) fl |= 3;
      } else {
        for (int c = tid; c < a.m; c += P) {
          int4 s0 = a.init[c];
          const int sb = (int)((sy[c >> 6] >> (c & 63)) & 1ull);
          fl |= sb | ((s0.z < 0 && sb) ? 2 : 0);   // bit 1: a check without edges can never be satisfied
          s0.w |= sb << 1;
          state[c] = make_float4(__int_as_float(s0.x), __int_as_float(s0.y), __int_as_float(s0.z),
                                 __int_as_float(s0.w));
        }
        for (int v = tid; v < a.n; v += P) L[v] = a.lam[v];
        for (int i = tid; i < (a.E4 >> 2); i += P) ((uint32_t*)sgn)[i] = a.sign0[i];
      }
      if (fl) atomicOr(&s_flag, fl);
    }
    __syncthreads();
    const int f0 = MULTI ? __builtin_amdgcn_readfirstlane(s_flag) : s_flag;
    int itr = 0;
    bool conv = true;
    if (f0 & 1) {
      conv = false;
      for (int t = 1;; ++t) {
        // variable pass: L^t from the state of iteration t
        if constexpr (PK && GSTATE) {
          // degree chunks: a column's first and last edge are on the same step
          // in every lane of the wave, so those branches are uniform (lane 0's
          // flags).  BP_AHEAD steps' loads go out before any of their stores (the
          // compiler cannot tell that L and the check states do not overlap);
          // records are read BP_AHEAD steps ahead.
          const float* wt = use_w ? a.w + (int64_t)(t - 1) * a.E : nullptr;
          float acc = 0.0f;
          int vo = tid;                                   // v' of the lane's current column
          const int32_t* rp = a.pvs4 + tid;
          const int32_t* ep = a.pve + tid;
          constexpr int U = GSTATE ? BP_AHEAD : 2;   // (LDS: two steps, fewer registers)
          int r[U];
          int ev[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            r[u] = rec(rp + (size_t)u * P);
            ev[u] = use_w ? rec(ep + (size_t)u * P) : 0;
          }
          for (int k = 0; k < a.Kv4; k += U) {
            float4 sv[U];
            float lv[U];
            int vu = vo;                                  // the column slot of step u
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int f = __builtin_amdgcn_readfirstlane(r[u]);
              sv[u] = ld_state(r[u] & R_IDX);
              lv[u] = (f & R_FIRST) ? gload(a.lamp + vu) : 0.0f;
              vu += (f & R_LAST) ? P : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int x = r[u], f = __builtin_amdgcn_readfirstlane(x);
              const int sh = (x >> R_SH) & 31;
              const float4 st = sv[u];
              const float at = use_w ? rec(wt + ev[u]) : a.alpha;
              const float mag = __fmul_rn(at, sh == __float_as_int(st.z) ? st.y : st.x);
              if (f & R_FIRST) acc = lv[u];               // lambda_v on a column's first edge
              acc = __fadd_rn(acc, ((__float_as_int(st.w) >> sh) & 1) ? -mag : mag);
              if (f & R_LAST) {
                st_L(vo, acc);
                vo += P;
              }
              r[u] = rec(rp + (size_t)(k + U + u) * P);
              if (use_w) ev[u] = rec(ep + (size_t)(k + U + u) * P);
            }
          }
        } else if constexpr (PK) {
          // state in LDS: per-lane flags, int2 records read two steps ahead (the
          // schedule holds two rows of padding past its even length)
          const float* wt = use_w ? a.w + (int64_t)(t - 1) * a.E : nullptr;
          float acc = 0.0f;
          int vo = tid;                                   // v' of the lane's current column
          // x: the record's flag word; lam = lambda_v (read on a column's first edge)
          auto vstep = [&](const int x, const float lam, const int e, const float4 s) {
            const int sh = (x >> R_SH) & 31;
            const float at = use_w ? rec(wt + e) : a.alpha;
            const float mag = __fmul_rn(at, sh == __float_as_int(s.z) ? s.y : s.x);
            const float base = (x & R_FIRST) ? lam : acc;   // lambda_v on a column's first edge
            acc = __fadd_rn(base, ((__float_as_int(s.w) >> sh) & 1) ? -mag : mag);
            if (x & R_LAST) {
              st_L(vo, acc);
              vo += P;
            }
          };
          const int32_t* ep = a.pve + tid;
          {
            const int2* rp = a.pvs + tid;
            int2 ra = rec(rp), rb = rec(rp + P);
            int ea = 0, eb = 0;
            if (use_w) { ea = rec(ep); eb = rec(ep + P); }
            for (int k = 0; k < a.Kv; k += 2) {
              vstep(ra.x, __int_as_float(ra.y), ea, state[ra.x & R_IDX]);
              ra = rec(rp + (size_t)(k + 2) * P);
              if (use_w) ea = rec(ep + (size_t)(k + 2) * P);
              vstep(rb.x, __int_as_float(rb.y), eb, state[rb.x & R_IDX]);
              rb = rec(rp + (size_t)(k + 3) * P);
              if (use_w) eb = rec(ep + (size_t)(k + 3) * P);
            }
          }
        } else {
          const float* wt = use_w ? a.w + (int64_t)(t - 1) * a.E : nullptr;
          float acc = 0.0f;
          auto vstep = [&](const int4 r) {
            const int v = r.x & R_IDX, e = r.y, c = r.z;
            const float4 s = ld_state(c);
            const float at = use_w ? rec(wt + (e < a.E32 ? e : 0)) : a.alpha;
            const float mag = __fmul_rn(at, e == __float_as_int(s.z) ? s.y : s.x);
            const int fl = __float_as_int(s.w);
            const float base = (r.x & R_FIRST) ? __int_as_float(r.w) : acc;   // lambda_v on a column's first edge
            acc = __fadd_rn(base, (((fl >> 1) ^ fl ^ sgn[e]) & 1) ? -mag : mag);
            if (r.x & R_LAST) st_L(v, acc);
          };
          // records are read two steps ahead; the schedule holds two rows of
          // padding past its (even) length, so every read is in bounds
          const int4* rp = a.vsched + tid;
          int4 ra = rec(rp), rb = rec(rp + P);
          for (int k = 0; k < a.Kv; k += 2) {
            vstep(ra);
            ra = rec(rp + (size_t)(k + 2) * P);
            vstep(rb);
            rb = rec(rp + (size_t)(k + 3) * P);
          }
        }
        __syncthreads();
        // check pass: H [L^t < 0] = s ?  and, if t < T, the state of iteration t + 1
        const bool update = t < a.T;
        int unsat = (f0 >> 1) & 1;
        {
          const float* wo = use_w ? a.w + (int64_t)(t - 1) * a.E : nullptr;   // weights of the messages m^t
          float n1o = 0.0f, n2o = 0.0f, n1 = BP_BIG, n2 = BP_BIG;
          int nago = -1, nag = -1, sc = 0, spo = 0, npar = 0, hard = 0;
          int flo = 0, nbits = 0;                        // PK: the old record's word, the new message signs
          // x: the record's flag word; e: the CSR edge (PK: for the weights only);
          // get_s() gives the check's state (called on a check's first edge only),
          // get_L() gives L_v
          auto cstep = [&](const int x, const int c, const int e, auto&& get_s, auto&& get_L) {
            const bool first = (x & R_FIRST) != 0;
            const int sh = (x >> R_SH) & 31;
            const int key = PK ? sh : e;                 // how the check state names its argmin edge
            // only lanes that start a check read its state (the others carry it)
            if (first) {
              const float4 s = get_s();
              const int fl = __float_as_int(s.w);
              n1o = s.x;
              n2o = s.y;
              nago = __float_as_int(s.z);
              sc = (fl >> 1) & 1;
              spo = fl & 1;
              flo = fl;
            }
            const float Lv = get_L();
            n1 = first ? BP_BIG : n1;
            n2 = first ? BP_BIG : n2;
            nag = first ? -1 : nag;
            npar = first ? 0 : npar;
            hard = (first ? 0 : hard) ^ (Lv < 0.0f ? 1 : 0);
            if (update) {
              const float ao = use_w ? rec(wo + (e < a.E32 ? e : 0)) : a.alpha;
              const float mag = __fmul_rn(ao, key == nago ? n2o : n1o);
              int neg;
              if constexpr (PK) neg = (flo >> sh) & 1;
              else neg = sc ^ spo ^ sgn[e];
              const float q = __fsub_rn(Lv, neg ? -mag : mag);   // q = L_v - m_old
              const float aq = fabsf(q);
              const int ng = q < 0.0f ? 1 : 0;
              const bool lt1 = aq < n1, lt2 = aq < n2;
              n2 = lt1 ? n1 : (lt2 ? aq : n2);
              n1 = lt1 ? aq : n1;
              nag = lt1 ? key : nag;
              npar ^= ng;
              if constexpr (PK) nbits = (first ? 0 : nbits) | (ng << sh);
              else sgn[e] = (uint8_t)ng;
            }
            if (x & R_LAST) {
              unsat |= hard != sc;
              if (update) {
                // PK: message sign of edge j = s_c + parity + sgn q_j (mod 2)
                const int w = PK ? ((sc << 1) | ((nbits ^ ((sc ^ npar) ? (int)0xFFFFFFFCu : 0)) & (int)0xFFFFFFFCu))
                                 : ((sc << 1) | npar);
                st_state(c, make_float4(n1, n2, __int_as_float(nag), __int_as_float(w)));
              }
            }
          };
          if constexpr (PK && GSTATE) {
            // degree chunks: a check's first and last edge are on the same step in
            // every lane of the wave, so those branches are uniform (lane 0's
            // flags) and the check states are read and written a whole wave at a
            // time.  BP_AHEAD steps' loads go out before any of their stores (a
            // lane's checks are distinct, so a store never feeds a later read of
            // the pass).
            const int32_t* rp = a.pcs4 + tid;
            const int32_t* ep = a.pce + tid;
            constexpr int U = GSTATE ? BP_AHEAD : 2;   // (LDS: two steps, fewer registers)
            int r[U];
            int ev[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              r[u] = rec(rp + (size_t)u * P);
              ev[u] = use_w ? rec(ep + (size_t)u * P) : 0;
            }
            int co = tid;                                 // the slot of the lane's current check
            for (int k = 0; k < a.Kc4; k += U) {
              float Lu[U];
              float4 sv[U];
              int cu[U];
#pragma unroll
              for (int u = 0; u < U; ++u) {
                const int f = __builtin_amdgcn_readfirstlane(r[u]);
                Lu[u] = ld_L(r[u] & R_IDX);
                cu[u] = co;
                sv[u] = (f & R_FIRST) ? ld_state(co) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                co += (f & R_LAST) ? P : 0;
              }
#pragma unroll
              for (int u = 0; u < U; ++u) {
                const int x = r[u], f = __builtin_amdgcn_readfirstlane(x);
                const int sh = (x >> R_SH) & 31;
                if (f & R_FIRST) {
                  const float4 st = sv[u];
                  n1o = st.x;
                  n2o = st.y;
                  nago = __float_as_int(st.z);
                  flo = __float_as_int(st.w);
                  sc = (flo >> 1) & 1;
                  n1 = BP_BIG;
                  n2 = BP_BIG;
                  nag = -1;
                  npar = 0;
                  hard = 0;
                  nbits = 0;
                }
                const float Lv = Lu[u];
                hard ^= Lv < 0.0f ? 1 : 0;
                if (update) {
                  const float ao = use_w ? rec(wo + ev[u]) : a.alpha;
                  const float mag = __fmul_rn(ao, sh == nago ? n2o : n1o);
                  const float q = __fsub_rn(Lv, ((flo >> sh) & 1) ? -mag : mag);   // q = L_v - m_old
                  const float aq = fabsf(q);
                  const int ng = q < 0.0f ? 1 : 0;
                  const bool lt1 = aq < n1, lt2 = aq < n2;
                  n2 = lt1 ? n1 : (lt2 ? aq : n2);
                  n1 = lt1 ? aq : n1;
                  nag = lt1 ? sh : nag;
                  npar ^= ng;
                  nbits |= ng << sh;
                }
                if (f & R_LAST) {
                  unsat |= hard != sc;
                  if (update) {
                    // message sign of edge j = s_c + parity + sgn q_j (mod 2)
                    const int w = (sc << 1) | ((nbits ^ ((sc ^ npar) ? (int)0xFFFFFFFCu : 0)) & (int)0xFFFFFFFCu);
                    st_state(cu[u], make_float4(n1, n2, __int_as_float(nag), __int_as_float(w)));
                  }
                }
                r[u] = rec(rp + (size_t)(k + U + u) * P);
                if (use_w) ev[u] = rec(ep + (size_t)(k + U + u) * P);
              }
            }
          } else if constexpr (PK) {
            // state in LDS: per-lane flags, int2 records read two steps ahead
            const int32_t* ep = a.pce + tid;
            {
              const int2* rp = a.pcs + tid;
              int2 ra = rec(rp), rb = rec(rp + P);
              int ea = 0, eb = 0;
              if (use_w) { ea = rec(ep); eb = rec(ep + P); }
              for (int k = 0; k < a.Kc; k += 2) {
                cstep(ra.x, ra.y, ea, [&] { return state[ra.y]; }, [&] { return L[ra.x & R_IDX]; });
                ra = rec(rp + (size_t)(k + 2) * P);
                if (use_w) ea = rec(ep + (size_t)(k + 2) * P);
                cstep(rb.x, rb.y, eb, [&] { return state[rb.y]; }, [&] { return L[rb.x & R_IDX]; });
                rb = rec(rp + (size_t)(k + 3) * P);
                if (use_w) eb = rec(ep + (size_t)(k + 3) * P);
              }
            }
          } else {
            const int4* rp = a.csched + tid;
            int4 ra = rec(rp), rb = rec(rp + P);
            for (int k = 0; k < a.Kc; k += 2) {
              cstep(ra.x, ra.z, ra.y, [&] { return ld_state(ra.z); }, [&] { return ld_L(ra.x & R_IDX); });
              ra = rec(rp + (size_t)(k + 2) * P);
              cstep(rb.x, rb.z, rb.y, [&] { return ld_state(rb.z); }, [&] { return ld_L(rb.x & R_IDX); });
              rb = rec(rp + (size_t)(k + 3) * P);
            }
          }
        }
        if (unsat) s_unsat[t & 1] = 1;                     // benign race: every writer stores 1
        if (tid == 0) s_unsat[(t + 1) & 1] = 0;            // read by every lane before the last barrier
        __syncthreads();
        if (!s_unsat[t & 1]) { itr = t; conv = true; break; }
        if (t >= a.T) { itr = a.T; break; }
      }
    }
    // finalise: prediction from the hard decision, or hand the posteriors to OSD
    if (tid == 0) s_pos = (!conv && a.use_osd) ? atomicAdd(&a.counters[2], 1) : -1;
    __syncthreads();
    const int pos = MULTI ? __builtin_amdgcn_readfirstlane(s_pos) : s_pos;
    uint64_t pm[MAX_OW] = {0ull, 0ull, 0ull, 0ull};
    for (int v = tid; v < a.n; v += P) {
      float Lv;
      if constexpr (PK) {
        const int vm = gload(a.vmap + v);
        Lv = (vm >= 0 && (f0 & 1)) ? ld_L(vm) : gload(a.lam + v);   // (no BP run: the priors)
      } else {
        Lv = L[v];
      }
      if (pos < 0 && Lv < 0.0f)
        for (int w = 0; w < a.ow; ++w) pm[w] ^= a.obs_mask[(int64_t)w * a.n + v];
      if (pos >= 0) a.osd_llr[(int64_t)pos * a.n + v] = Lv;
      if (a.llr) a.llr[shot * a.n + v] = Lv;
      if (a.ehat && pos < 0) a.ehat[shot * a.n + v] = Lv < 0.0f ? 1 : 0;
    }
    for (int w = 0; w < a.ow; ++w)
      if (pm[w]) atomicXor(&s_pm[w], (unsigned long long)pm[w]);
    __syncthreads();
    if (tid == 0) {
      if (pos < 0)
        for (int w = 0; w < a.ow; ++w) write_pred(a.pred, a.stride, a.nobs, shot, s_pm[w], w);
      else a.osd_queue[pos] = (int32_t)ls;
      if (a.iters) a.iters[shot] = itr;
      if (a.flags) a.flags[shot] = (uint8_t)((conv ? 1 : 0) | (pos >= 0 ? 2 : 0));
      c_nontriv += (itr > 0 || !conv) ? 1 : 0;
      c_conv += conv ? 1 : 0;
      c_osd += pos >= 0 ? 1 : 0;
      c_iters += (unsigned long long)itr;
      s_hist[itr < TMCS_BP_HIST_BINS - 1 ? itr : TMCS_BP_HIST_BINS - 1] += 1ull;
    }
  }
  if constexpr (!MULTI) flush();
}


template <typename T>
tmcs_status upload(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
  if (hipMalloc((void**)dst, bytes) != hipSuccess) return fail(TMCS_ENOMEM, "hipMalloc failed (dem)");
  if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(TMCS_EDEVICE, "hipMemcpy failed (dem)");
  return TMCS_OK;
}

template <typename T>
tmcs_status grow(T** p, size_t* cap, size_t need) {
  if (*cap >= need) return TMCS_OK;
  hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipMalloc((void**)p, need * sizeof(T)) != hipSuccess) return fail(TMCS_ENOMEM, "hipMalloc failed (decoder scratch)");
  *cap = need;
  return TMCS_OK;
}

void free_device(DecodeDevice* d) {
  hipFree(d->row_ptr); hipFree(d->col_idx); hipFree(d->col_ptr); hipFree(d->csc_row); hipFree(d->csc_edge);
  hipFree(d->lam); hipFree(d->obs_mask); hipFree(d->counters); hipFree(d->queue); hipFree(d->osd_queue);
  hipFree(d->osd_llr); hipFree(d->basis); hipFree(d->synd); hipFree(d->gstate); hipFree(d->init); hipFree(d->sign0);
  hipFree(d->rowmap); hipFree(d->retry); hipFree(d->lone);
  for (auto& q : d->scheds) {
    hipFree(q.c); hipFree(q.v); hipFree(q.f);
    hipFree(q.pce); hipFree(q.pve); hipFree(q.vmap);
    hipFree(q.pcL); hipFree(q.pvL); hipFree(q.pceL); hipFree(q.pveL); hipFree(q.vmapL); hipFree(q.corigL); hipFree(q.pinitL);
    hipFree(q.pc4); hipFree(q.pv4); hipFree(q.corig4); hipFree(q.pinit4); hipFree(q.lamp);
  }
  *d = DecodeDevice();
}

tmcs_status build_state(const Dem& D, int dev, DecodeDevice** out) {
  DecodeDevice* d = new DecodeDevice();
  d->device = dev;
  std::vector<int32_t> csc_row(D.row_idx.begin(), D.row_idx.end());
  std::vector<float> lam(D.cols);
  for (int j = 0; j < D.cols; ++j) lam[j] = (float)std::log((1.0 - D.priors[j]) / D.priors[j]);
  // observable masks word-major on the device ([ow][n]), so lanes of a wave read consecutive columns
  std::vector<uint64_t> obs_wm((size_t)D.obs_words * D.cols);
  for (int j = 0; j < D.cols; ++j)
    for (int w = 0; w < D.obs_words; ++w) obs_wm[(size_t)w * D.cols + j] = D.obs_mask[(size_t)j * D.obs_words + w];
  tmcs_status st;
  if ((st = upload(&d->row_ptr, D.row_ptr)) != TMCS_OK || (st = upload(&d->col_idx, D.col_idx)) != TMCS_OK ||
      (st = upload(&d->col_ptr, D.col_ptr)) != TMCS_OK || (st = upload(&d->csc_row, csc_row)) != TMCS_OK ||
      (st = upload(&d->csc_edge, D.csc_edge)) != TMCS_OK || (st = upload(&d->lam, lam)) != TMCS_OK ||
      (st = upload(&d->obs_mask, obs_wm)) != TMCS_OK) {
    free_device(d);
    delete d;
    return st;
  }
  // iteration 1 of BP has q_{v->c} = lambda_v: its check state and edge signs
  // follow from the DEM alone (same FP32 comparisons as the check pass)
  std::vector<int4> init(std::max(D.rows, 0)), init_pk(std::max(D.rows, 0));
  d->E4 = (int32_t)((D.edges + 3) & ~3ll);
  std::vector<uint8_t> sg((size_t)d->E4, 0);
  for (int c = 0; c < D.rows; ++c) {
    float n1 = BP_BIG, n2 = BP_BIG;
    int nag = -1, npar = 0;
    for (int32_t e = D.row_ptr[c]; e < D.row_ptr[c + 1]; ++e) {
      const float q = lam[D.col_idx[e]];
      const float aq = std::fabs(q);
      const int ng = q < 0.0f ? 1 : 0;
      if (aq < n1) { n2 = n1; n1 = aq; nag = e; }
      else if (aq < n2) { n2 = aq; }
      npar ^= ng;
      sg[e] = (uint8_t)ng;
    }
    int4 r;
    std::memcpy(&r.x, &n1, 4);
    std::memcpy(&r.y, &n2, 4);
    r.z = nag;
    r.w = npar;
    init[c] = r;
    d->max_row_deg = std::max(d->max_row_deg, D.row_ptr[c + 1] - D.row_ptr[c]);
    // packed: the sign of the message to the j-th edge in bit 2 + j (s_c = 0),
    // the argmin edge as 2 + its position
    uint32_t pw = 0;
    for (int32_t e = D.row_ptr[c]; e < D.row_ptr[c + 1] && e - D.row_ptr[c] < PK_MAX_DEG; ++e)
      pw |= (uint32_t)(npar ^ sg[e]) << (2 + e - D.row_ptr[c]);
    r.z = nag < 0 ? -1 : 2 + (nag - D.row_ptr[c]);
    r.w = (int32_t)pw;
    init_pk[c] = r;
  }
  if (d->max_row_deg <= PK_MAX_DEG && D.cols < R_IDX && D.rows < R_IDX) d->init_pk = init_pk;
  // checks without edges (a shot with such a detection event never satisfies
  // H e = s) and the observables flipped by the hard decision of lambda alone
  std::vector<uint64_t> lone((size_t)std::max((D.rows + 63) / 64, 1), 0ull);
  bool any_lone = false;
  for (int c = 0; c < D.rows; ++c)
    if (D.row_ptr[c + 1] == D.row_ptr[c]) { lone[c >> 6] |= 1ull << (c & 63); any_lone = true; }
  for (int j = 0; j < D.cols; ++j)
    if (lam[j] < 0.0f)
      for (int w = 0; w < D.obs_words && w < MAX_OW; ++w) {
        d->pm_lam[w] ^= D.obs_mask[(size_t)j * D.obs_words + w];
        if (D.col_ptr[j + 1] == D.col_ptr[j]) d->pm_iso[w] ^= D.obs_mask[(size_t)j * D.obs_words + w];
      }
  if (any_lone && (st = upload(&d->lone, lone)) != TMCS_OK) {
    free_device(d);
    delete d;
    return st;
  }
  std::vector<uint32_t> sg32((size_t)d->E4 / 4);
  if (!sg32.empty()) std::memcpy(sg32.data(), sg.data(), sg.size());
  if ((st = upload(&d->init, init)) != TMCS_OK || (st = upload(&d->sign0, sg32)) != TMCS_OK) {
    free_device(d);
    delete d;
    return st;
  }
  if (hipMalloc((void**)&d->counters, 8 * sizeof(int32_t)) != hipSuccess) {
    free_device(d);
    delete d;
    return fail(TMCS_ENOMEM, "hipMalloc failed (counters)");
  }
  *out = d;
  return TMCS_OK;
}

// Longest-processing-time assignment of items (checks or columns) of given
// sizes to P lanes; returns per-lane item lists (ascending) and the max load.
int lpt_assign(const std::vector<int>& size, int P, std::vector<std::vector<int>>* lanes) {
  std::vector<int> order(size.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return size[a] > size[b]; });
  lanes->assign(P, {});
  std::vector<std::pair<long, int>> heap;   // (load, lane), min-heap
  for (int l = 0; l < P; ++l) heap.push_back({0, l});
  auto cmp = [](const std::pair<long, int>& a, const std::pair<long, int>& b) { return a > b; };
  std::make_heap(heap.begin(), heap.end(), cmp);
  for (int it : order) {
    if (size[it] == 0) continue;
    std::pop_heap(heap.begin(), heap.end(), cmp);
    auto& top = heap.back();
    (*lanes)[top.second].push_back(it);
    top.first += size[it];
    std::push_heap(heap.begin(), heap.end(), cmp);
  }
  long kmax = 0;
  for (auto& h : heap) kmax = std::max(kmax, h.first);
  for (auto& l : *lanes) std::sort(l.begin(), l.end());
  return (int)kmax;
}

// Strided assignment: lane l takes items l, l + P, l + 2P, ...  At a given step
// the lanes of a wave are on consecutive items, so their state reads are
// coalesced (whole cache lines of consecutive checks or columns); loads differ
// between lanes by the degree variation only.  Returns the max load.
int strided_assign(const std::vector<int>& size, int P, std::vector<std::vector<int>>* lanes) {
  lanes->assign(P, {});
  std::vector<long> load(P, 0);
  int j = 0;
  for (size_t i = 0; i < size.size(); ++i) {
    if (size[i] == 0) continue;
    (*lanes)[j].push_back((int)i);
    load[j] += size[i];
    j = (j + 1) % P;
  }
  long kmax = 0;
  for (long x : load) kmax = std::max(kmax, x);
  return (int)kmax;
}

// Schedules of the check and variable passes for team size P and assignment
// (cfg.bp_sched: 1 longest-processing-time lists, 2 strided), cached per both.
// (Contiguous per-lane ranges were also tried for state in device memory: the
// lanes of a step then sit a fixed stride apart and hit the same HBM channels,
// 7x slower.)  P < 64 builds the lists of the lanes kernel, one per wave, each
// stored contiguously ([P][K + LANES_UNROLL]): their length is a multiple of
// LANES_UNROLL, followed by LANES_UNROLL records of padding.  Team lists are
// interleaved ([K + 2][P]): even length, two rows of padding.
// Record bits of an edge's position j within its check (packed check state).
int32_t pos_bits(int32_t j) { return j < PK_MAX_DEG ? (2 + j) << R_SH : 0; }

tmcs_status get_sched(const Dem& D, DecodeDevice* d, int P, int mode, DecodeDevice::Sched* out) {
  for (const auto& q : d->scheds)
    if (q.P == P && q.mode == mode) { *out = q; return TMCS_OK; }
  DecodeDevice::Sched q;
  q.P = P;
  q.mode = mode;
  auto assign = mode == 2 ? strided_assign : lpt_assign;
  std::vector<std::vector<int>> lanes;
  std::vector<int> rdeg(std::max(D.rows, 0)), cdeg(std::max(D.cols, 0));
  for (int c = 0; c < D.rows; ++c) rdeg[c] = D.row_ptr[c + 1] - D.row_ptr[c];
  for (int v = 0; v < D.cols; ++v) cdeg[v] = D.col_ptr[v + 1] - D.col_ptr[v];
  // padding steps touch only spare LDS slots (edge E4, check m) and never
  // carry FIRST/LAST, so their results are never stored
  const int4 pad = make_int4(0, d->E4, D.rows, 0);
  // K is rounded up to the batch (team lists: even), plus one batch of padding read by the prefetch
  const int kb = P < 64 ? LANES_UNROLL : 2;
  auto round_k = [&](int k) { return (k + kb - 1) / kb * kb; };
  q.Kc = round_k(assign(rdeg, P, &lanes));
  std::vector<int4> cs((size_t)(q.Kc + kb) * P, pad);
  for (int l = 0; l < P; ++l) {
    int k = 0;
    for (int c : lanes[l])
      for (int32_t e = D.row_ptr[c]; e < D.row_ptr[c + 1]; ++e, ++k) {
        int32_t x = D.col_idx[e] | pos_bits(e - D.row_ptr[c]);
        if (e == D.row_ptr[c]) x |= R_FIRST;
        if (e == D.row_ptr[c + 1] - 1) x |= R_LAST;
        cs[P < 64 ? (size_t)l * (q.Kc + kb) + k : (size_t)k * P + l] = make_int4(x, e, c, 0);
      }
  }
  q.Kv = round_k(assign(cdeg, P, &lanes));
  std::vector<int4> vs((size_t)(q.Kv + kb) * P, pad);
  for (int l = 0; l < P; ++l) {
    int k = 0;
    for (int v : lanes[l])
      for (int32_t j = D.col_ptr[v]; j < D.col_ptr[v + 1]; ++j, ++k) {
        int32_t x = v | pos_bits(D.csc_edge[j] - D.row_ptr[D.row_idx[j]]);
        if (j == D.col_ptr[v]) x |= R_FIRST;
        if (j == D.col_ptr[v + 1] - 1) x |= R_LAST;
        float lv = (float)std::log((1.0 - D.priors[v]) / D.priors[v]);
        int32_t lbits;
        std::memcpy(&lbits, &lv, 4);
        vs[P < 64 ? (size_t)l * (q.Kv + kb) + k : (size_t)k * P + l] = make_int4(x, D.csc_edge[j], D.row_idx[j], lbits);
      }
  }
  tmcs_status st;
  if ((st = upload(&q.c, cs)) != TMCS_OK) return st;
  if ((st = upload(&q.v, vs)) != TMCS_OK) { hipFree(q.c); return st; }
  d->scheds.push_back(q);
  *out = q;
  return TMCS_OK;
}

// Records of the single-pass kernel for team size P: the check-pass lane lists
// of get_sched (same assignment), two int4 per edge ([K + 2][P][2]).
tmcs_status get_fsched(const Dem& D, DecodeDevice* d, int P, int mode, DecodeDevice::Sched* out) {
  tmcs_status st = get_sched(D, d, P, mode, out);
  if (st != TMCS_OK) return st;
  DecodeDevice::Sched* q = nullptr;
  for (auto& x : d->scheds)
    if (x.P == P && x.mode == mode) q = &x;
  if (!q) return fail(TMCS_EDEVICE, "BP schedule cache");
  if (q->f) { *out = *q; return TMCS_OK; }
  std::vector<int4> cs((size_t)(q->Kc + 2) * P);
  if (hipMemcpy(cs.data(), q->c, cs.size() * sizeof(int4), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(TMCS_EDEVICE, "hipMemcpy failed (BP schedule)");
  // per CSR edge: its column, and where that column's entries start in CSC order
  std::vector<int32_t> pos_in_col((size_t)std::max<int64_t>(D.edges, 1));
  for (int v = 0; v < D.cols; ++v)
    for (int32_t j = D.col_ptr[v]; j < D.col_ptr[v + 1]; ++j) pos_in_col[D.csc_edge[j]] = j;
  std::vector<int4> fs((size_t)(q->Kc + 2) * P * 2);
  for (size_t i = 0; i < cs.size(); ++i) {
    const int4 r = cs[i];
    int4 A = r, B = make_int4(-1, 0, 0, 0);
    if (r.y < D.edges && r.z < D.rows) {               // (padding records keep B = degree 1, no flags)
      const int v = r.x & R_IDX, e = r.y, c = r.z;
      const int32_t j0 = D.col_ptr[v], deg = D.col_ptr[v + 1] - j0;
      float lv = (float)std::log((1.0 - D.priors[v]) / D.priors[v]);
      std::memcpy(&A.w, &lv, 4);
      const int firstcol = D.row_idx[j0] == c ? 2 : 0;
      if (deg == 2) {
        const int32_t jo = pos_in_col[e] == j0 ? j0 + 1 : j0;
        const int c2 = D.row_idx[jo];
        B = make_int4(c2, D.csc_edge[jo], (c2 < c ? 1 : 0) | firstcol, 0);
      } else if (deg == 1) {
        B = make_int4(-1, 0, firstcol, 0);
      } else {
        B = make_int4(-2, j0, firstcol, deg);
      }
    }
    fs[2 * i] = A;
    fs[2 * i + 1] = B;
  }
  if ((st = upload(&q->f, fs)) != TMCS_OK) return st;
  q->Kf = q->Kc;
  *out = *q;
  return TMCS_OK;
}

// Records of the packed-state team kernel with its state in LDS, for team size
// P: the longest-processing-time lane lists of get_sched; checks numbered in the
// order the lanes first reach them (step i of lane l before step i of lane
// l + 1, before step i + 1), the i-th column of lane l at v' = i P + l; int2
// records {v' | position | flags, c'} and {c' | position | flags, lambda_v}.
// (The degree chunks of get_psched pad small DEMs too much: on the d = 5 and
// d = 11 surface-code DEMs they made this kernel 23-29 % slower.)
tmcs_status get_psched_lds(const Dem& D, DecodeDevice* d, int P, int mode, DecodeDevice::Sched* out) {
  tmcs_status st = get_sched(D, d, P, mode, out);
  if (st != TMCS_OK) return st;
  DecodeDevice::Sched* q = nullptr;
  for (auto& x : d->scheds)
    if (x.P == P && x.mode == mode) q = &x;
  if (!q) return fail(TMCS_EDEVICE, "BP schedule cache");
  if (q->pcL) { *out = *q; return TMCS_OK; }
  if (d->init_pk.empty()) return fail(TMCS_EUNSUPPORTED, "packed BP state: a check has more than 30 edges");
  auto assign = mode == 2 ? strided_assign : lpt_assign;
  std::vector<int> rdeg(std::max(D.rows, 0)), cdeg(std::max(D.cols, 0));
  for (int c = 0; c < D.rows; ++c) rdeg[c] = D.row_ptr[c + 1] - D.row_ptr[c];
  for (int v = 0; v < D.cols; ++v) cdeg[v] = D.col_ptr[v + 1] - D.col_ptr[v];
  std::vector<std::vector<int>> rl, cl;
  assign(rdeg, P, &rl);
  assign(cdeg, P, &cl);
  size_t ri = 0, ci = 0;
  for (int l = 0; l < P; ++l) { ri = std::max(ri, rl[l].size()); ci = std::max(ci, cl[l].size()); }
  std::vector<int32_t> cslot(std::max(D.rows, 0), -1), corig, vmap(std::max(D.cols, 0), -1);
  for (size_t i = 0; i < ri; ++i)
    for (int l = 0; l < P; ++l)
      if (i < rl[l].size()) { cslot[rl[l][i]] = (int32_t)corig.size(); corig.push_back(rl[l][i]); }
  for (int l = 0; l < P; ++l)
    for (size_t i = 0; i < cl[l].size(); ++i) vmap[cl[l][i]] = (int32_t)(i * P + l);
  const int32_t Mpk = (int32_t)corig.size(), Npk = (int32_t)(ci * P);
  if (Npk > R_IDX) return fail(TMCS_EUNSUPPORTED, "BP: too many column slots");
  // padding steps read the spare slots (check Mpk, column Npk) and never store;
  // the lists hold two rows of padding past their (even) length
  std::vector<int2> pc((size_t)(q->Kc + 2) * P, make_int2(Npk, Mpk)), pv((size_t)(q->Kv + 2) * P, make_int2(Mpk, 0));
  std::vector<int32_t> pce(pc.size(), 0), pve(pv.size(), 0);
  for (int l = 0; l < P; ++l) {
    size_t k = 0;
    for (int c : rl[l])
      for (int32_t e = D.row_ptr[c]; e < D.row_ptr[c + 1]; ++e, ++k) {
        int32_t x = vmap[D.col_idx[e]] | pos_bits(e - D.row_ptr[c]);
        if (e == D.row_ptr[c]) x |= R_FIRST;
        if (e == D.row_ptr[c + 1] - 1) x |= R_LAST;
        pc[k * P + l] = make_int2(x, cslot[c]);
        pce[k * P + l] = e;
      }
    k = 0;
    for (int v : cl[l]) {
      const float lv = (float)std::log((1.0 - D.priors[v]) / D.priors[v]);
      int32_t lbits;
      std::memcpy(&lbits, &lv, 4);
      for (int32_t j = D.col_ptr[v]; j < D.col_ptr[v + 1]; ++j, ++k) {
        const int c = D.row_idx[j], e = D.csc_edge[j];
        int32_t f = pos_bits(e - D.row_ptr[c]);
        if (j == D.col_ptr[v]) f |= R_FIRST;
        if (j == D.col_ptr[v + 1] - 1) f |= R_LAST;
        pv[k * P + l] = make_int2(cslot[c] | f, lbits);
        pve[k * P + l] = e;
      }
    }
  }
  std::vector<int4> pinit(std::max<int32_t>(Mpk, 1));
  for (int32_t c = 0; c < Mpk; ++c) pinit[c] = d->init_pk[corig[c]];
  if (corig.empty()) corig.push_back(0);
  if (vmap.empty()) vmap.push_back(-1);
  // (pcL last: a schedule with pcL set is complete)
  if ((st = upload(&q->pvL, pv)) != TMCS_OK || (st = upload(&q->pceL, pce)) != TMCS_OK ||
      (st = upload(&q->pveL, pve)) != TMCS_OK || (st = upload(&q->vmapL, vmap)) != TMCS_OK ||
      (st = upload(&q->corigL, corig)) != TMCS_OK || (st = upload(&q->pinitL, pinit)) != TMCS_OK ||
      (st = upload(&q->pcL, pc)) != TMCS_OK)
    return st;
  q->MpkL = Mpk;
  q->NpkL = Npk;
  *out = *q;
  return TMCS_OK;
}

// Records of the packed-state team kernel with its state in device memory, for
// team size P.  The checks with
// edges are sorted by (degree, index) and cut into chunks of 64, one check per
// lane of a wave, and the chunks go to the P / 64 waves in turn; the columns
// likewise.  A chunk takes as many steps as its largest degree: shorter checks
// (columns) and empty lanes get no-op edges, so a check's (column's) first and
// last edge fall on the same step in every lane of a wave and the kernel
// branches on them uniformly.  Lane l's k-th check is at slot c' = k P + l and
// its k-th column at v' = k P + l.  No-op edges: in the check pass they read
// L slot Npk (+BIG in every shot: q stays +BIG, so the minima, the sign parity
// and the hard decision do not change); in the variable pass they read check
// slot Mpk + 1 (n1 = n2 = +0, every message sign set: the message is -0, and
// x + (-0) = x for every x).  Empty check slots start with s_c = 0 and are
// only ever read by their own no-op check.
tmcs_status get_psched(const Dem& D, DecodeDevice* d, int P, int mode, DecodeDevice::Sched* out) {
  tmcs_status st = get_sched(D, d, P, mode, out);
  if (st != TMCS_OK) return st;
  DecodeDevice::Sched* q = nullptr;
  for (auto& x : d->scheds)
    if (x.P == P && x.mode == mode) q = &x;
  if (!q) return fail(TMCS_EDEVICE, "BP schedule cache");
  if (q->pc4) { *out = *q; return TMCS_OK; }
  if (d->init_pk.empty()) return fail(TMCS_EUNSUPPORTED, "packed BP state: a check has more than 30 edges");
  if (P % 64) return fail(TMCS_EINVAL, "packed BP state: team size must be a multiple of 64");
  const int NW = P / 64;
  std::vector<int> rdeg(std::max(D.rows, 0)), cdeg(std::max(D.cols, 0));
  for (int c = 0; c < D.rows; ++c) rdeg[c] = D.row_ptr[c + 1] - D.row_ptr[c];
  for (int v = 0; v < D.cols; ++v) cdeg[v] = D.col_ptr[v + 1] - D.col_ptr[v];
  // chunks of 64 items (-1: an empty lane) in (degree, index) order, and their widths
  auto make_chunks = [](const std::vector<int>& deg, std::vector<std::vector<int>>* ch, std::vector<int>* width) {
    std::vector<int> items;
    for (int i = 0; i < (int)deg.size(); ++i)
      if (deg[i] > 0) items.push_back(i);
    std::stable_sort(items.begin(), items.end(), [&](int a, int b) { return deg[a] < deg[b]; });
    for (size_t i = 0; i < items.size(); i += 64) {
      std::vector<int> c(64, -1);
      int w = 0;
      for (size_t j = 0; j < 64 && i + j < items.size(); ++j) {
        c[j] = items[i + j];
        w = std::max(w, deg[items[i + j]]);
      }
      ch->push_back(c);
      width->push_back(w);
    }
  };
  std::vector<std::vector<int>> cch, vch;
  std::vector<int> cw, vw;
  make_chunks(rdeg, &cch, &cw);
  make_chunks(cdeg, &vch, &vw);
  // chunk i goes to wave i mod NW, as its (i / NW)-th; steps per wave
  auto steps = [&](const std::vector<int>& width) {
    int kmax = 0;
    for (int w = 0; w < NW; ++w) {
      int k = 0;
      for (size_t i = w; i < width.size(); i += NW) k += width[i];
      kmax = std::max(kmax, k);
    }
    return kmax;
  };
  const int Kc = steps(cw), Kv = steps(vw);
  const int32_t Kc4 = (Kc + BP_AHEAD - 1) / BP_AHEAD * BP_AHEAD, Kv4 = (Kv + BP_AHEAD - 1) / BP_AHEAD * BP_AHEAD;
  const int32_t Mpk4 = (int32_t)((cch.size() + NW - 1) / NW) * P, Npk = (int32_t)((vch.size() + NW - 1) / NW) * P;
  if (Npk + 1 > R_IDX || Mpk4 + 2 > R_IDX) return fail(TMCS_EUNSUPPORTED, "BP: too many column or check slots");
  const int32_t SINK = Mpk4 + 1;
  std::vector<int32_t> cslot(std::max(D.rows, 0), -1), vmap(std::max(D.cols, 0), -1);
  std::vector<int32_t> corig4((size_t)Mpk4 + 2, -1);
  for (size_t i = 0; i < cch.size(); ++i)
    for (int j = 0; j < 64; ++j)
      if (cch[i][j] >= 0) {
        const int32_t slot = (int32_t)((i / NW) * P + (i % NW) * 64 + j);
        cslot[cch[i][j]] = slot;
        corig4[slot] = cch[i][j];
      }
  for (size_t i = 0; i < vch.size(); ++i)
    for (int j = 0; j < 64; ++j)
      if (vch[i][j] >= 0) vmap[vch[i][j]] = (int32_t)((i / NW) * P + (i % NW) * 64 + j);
  // records; the rows past a wave's last chunk carry no flags and are never stored
  std::vector<int32_t> pc4((size_t)(Kc4 + BP_AHEAD) * P, Npk), pv4((size_t)(Kv4 + BP_AHEAD) * P, Mpk4);
  std::vector<int32_t> pce(pc4.size(), 0), pve(pv4.size(), 0);
  std::vector<float> lamp((size_t)Npk + 1, 0.0f);
  for (int w = 0; w < NW; ++w) {
    size_t k = 0;
    for (size_t i = w; i < cch.size(); i += NW)
      for (int sx = 0; sx < cw[i]; ++sx, ++k) {
        const int32_t f = (sx == 0 ? R_FIRST : 0) | (sx == cw[i] - 1 ? R_LAST : 0);
        for (int j = 0; j < 64; ++j) {
          const int c = cch[i][j];
          const size_t at = k * P + w * 64 + j;
          if (c >= 0 && sx < rdeg[c]) {
            const int32_t e = D.row_ptr[c] + sx;
            pc4[at] = vmap[D.col_idx[e]] | pos_bits(sx) | f;
            pce[at] = e;
          } else {
            pc4[at] = Npk | pos_bits(sx) | f;              // no-op edge
          }
        }
      }
    k = 0;
    for (size_t i = w; i < vch.size(); i += NW)
      for (int sx = 0; sx < vw[i]; ++sx, ++k) {
        const int32_t f = (sx == 0 ? R_FIRST : 0) | (sx == vw[i] - 1 ? R_LAST : 0);
        for (int j = 0; j < 64; ++j) {
          const int v = vch[i][j];
          const size_t at = k * P + w * 64 + j;
          if (v >= 0 && sx < cdeg[v]) {
            const int32_t jj = D.col_ptr[v] + sx;
            const int c = D.row_idx[jj], e = D.csc_edge[jj];
            pv4[at] = cslot[c] | pos_bits(e - D.row_ptr[c]) | f;
            pve[at] = e;
          } else {
            pv4[at] = SINK | f;                            // no-op edge (message -0)
          }
        }
      }
  }
  for (int v = 0; v < D.cols; ++v)
    if (vmap[v] >= 0) lamp[vmap[v]] = (float)std::log((1.0 - D.priors[v]) / D.priors[v]);
  // check slots: the iteration-1 state of a real check; empty and padding slots
  // s_c = 0 with no minima; the sink the no-op message state
  int4 empty;
  {
    const float big = BP_BIG;
    std::memcpy(&empty.x, &big, 4);
    std::memcpy(&empty.y, &big, 4);
    empty.z = -1;
    empty.w = 0;
  }
  std::vector<int4> pinit4((size_t)Mpk4 + 2, empty);
  for (int32_t c = 0; c < Mpk4; ++c)
    if (corig4[c] >= 0) pinit4[c] = d->init_pk[corig4[c]];
  pinit4[SINK] = make_int4(0, 0, -1, -1);                  // +0, +0, no argmin, every sign set
  if (vmap.empty()) vmap.push_back(-1);
  // (pc4 last: a schedule with pc4 set is complete)
  if ((st = upload(&q->pv4, pv4)) != TMCS_OK || (st = upload(&q->pce, pce)) != TMCS_OK ||
      (st = upload(&q->pve, pve)) != TMCS_OK || (st = upload(&q->vmap, vmap)) != TMCS_OK ||
      (st = upload(&q->corig4, corig4)) != TMCS_OK || (st = upload(&q->pinit4, pinit4)) != TMCS_OK ||
      (st = upload(&q->lamp, lamp)) != TMCS_OK || (st = upload(&q->pc4, pc4)) != TMCS_OK)
    return st;
  q->Mpk4 = Mpk4;
  q->Npk = Npk;
  q->Kc4 = Kc4;
  q->Kv4 = Kv4;
  *out = *q;
  return TMCS_OK;
}

// The device state cached on the DEM handle (rebuilt when the device changes).
tmcs_status ensure_device(const Dem& dc, DecodeDevice** out) {
  Dem& D = const_cast<Dem&>(dc);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TMCS_EDEVICE, "no HIP device");
  DecodeDevice* d = (DecodeDevice*)D.device;
  if (d && d->device == dev) { *out = d; return TMCS_OK; }
  if (d) { free_device(d); delete d; D.device = nullptr; }
  tmcs_status st = build_state(D, dev, &d);
  if (st != TMCS_OK) return st;
  D.device = d;
  *out = d;
  return TMCS_OK;
}

int device_cus() {
  int dev = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus > 0 ? cus : 256;
}


// Dynamic LDS beyond 64 KB for every LDS-state variant of k_bp.
bool bp_lds_allow(size_t lds) {
  const void* f[] = {(const void*)k_bp<false, false, false, false>, (const void*)k_bp<true, false, false, false>,
                     (const void*)k_bp<false, false, true, false>,  (const void*)k_bp<true, false, true, false>,
                     (const void*)k_bp<false, false, false, true>,  (const void*)k_bp<true, false, false, true>,
                     (const void*)k_bp<false, false, true, true>,   (const void*)k_bp<true, false, true, true>};
  for (const void* p : f)
    if (hipFuncSetAttribute(p, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return false;
  return true;
}

// Launch of the team kernel variant (state in LDS: "k_bp", in device memory: "k_bp_dev").
template <bool MULTI>
void launch_k_bp(bool weighted, bool gstate, bool pk, int grid, int P, size_t lds, hipStream_t stream,
                 const BPArgs& a, const BPMulti& mu) {
  const dim3 g((unsigned)grid), b((unsigned)P);
  if (gstate) {
    if (pk) {
      if (weighted) TMCS_LAUNCH("k_bp_dev", (k_bp<true, true, MULTI, true>), g, b, 0, stream, a, mu);
      else TMCS_LAUNCH("k_bp_dev", (k_bp<false, true, MULTI, true>), g, b, 0, stream, a, mu);
    } else {
      if (weighted) TMCS_LAUNCH("k_bp_dev", (k_bp<true, true, MULTI, false>), g, b, 0, stream, a, mu);
      else TMCS_LAUNCH("k_bp_dev", (k_bp<false, true, MULTI, false>), g, b, 0, stream, a, mu);
    }
  } else {
    if (pk) {
      if (weighted) TMCS_LAUNCH("k_bp", (k_bp<true, false, MULTI, true>), g, b, lds, stream, a, mu);
      else TMCS_LAUNCH("k_bp", (k_bp<false, false, MULTI, true>), g, b, lds, stream, a, mu);
    } else {
      if (weighted) TMCS_LAUNCH("k_bp", (k_bp<true, false, MULTI, false>), g, b, lds, stream, a, mu);
      else TMCS_LAUNCH("k_bp", (k_bp<false, false, MULTI, false>), g, b, lds, stream, a, mu);
    }
  }
}

constexpr int64_t DECODE_CHUNK_MIN = 4096;

// Everything one decoder pass needs: launch shapes, scratch and the kernel
// arguments (filled by decode_prepare, used by the stage / BP / OSD launchers).
struct DecodePass {
  DecodeDevice* d = nullptr;
  const Dem* D = nullptr;
  tmcs_decoder_cfg cfg{};
  int64_t stride = 0;          // words per row of det / pred
  int64_t chunk = 0;           // shots per pass
  bool full = false;           // per-shot outputs requested (no compaction)
  int mw = 0;
  bool gstate = false;
  bool lanes = false;          // state in device memory, 64 shots per workgroup (bp_lanes.hip)
  bool fused = false;          // state in device memory, one pass per iteration (bp_fused.hip)
  bool pk = false;             // team kernel with the packed check state (no sign bytes)
  int P = 0, bp_grid_max = 0;
  size_t bp_lds = 0, team_bytes = 0;
  DecodeDevice::Sched sch;
  bool osd_win = false, osd_pfx = false, osd_bl = false;
  bool win2 = false;           // windowed: a smaller first window, then the full one on what it leaves open
  int npad = 0, pfx_keys = 0, pfx_rank = 0, osd_grid = 0, pfx_grid = 0, win1_grid = 0, win1_rows = 0;
  int win1_mw = 0;             // words of local rows of the first window (WIN_SMALL_MW or WIN_MID_MW)
  size_t osd_lds = 0, pfx_lds = 0, win1_lds = 0;
};

// Expected number of detection events per shot: sum over detectors of the
// probability that an odd number of its mechanisms fire.
double expected_events(const Dem& D) {
  double ev = 0.0;
  for (int c = 0; c < D.rows; ++c) {
    double prod = 1.0;
    for (int32_t e = D.row_ptr[c]; e < D.row_ptr[c + 1]; ++e) prod *= 1.0 - 2.0 * D.priors[D.col_idx[e]];
    ev += 0.5 * (1.0 - prod);
  }
  return ev;
}

// Workgroups of a lanes launch over ns shots: one per 64 shots, at most the
// resident grid, and at most LANES_SLAB_MAX bytes of state in device memory.
constexpr size_t LANES_SLAB_MAX = 48ull << 30;
int lanes_grid(int grid_max, size_t slab, int64_t ns) {
  const int64_t groups = (std::max<int64_t>(ns, 1) + 63) / 64;
  const int64_t by_mem = std::max<int64_t>(1, (int64_t)(LANES_SLAB_MAX / std::max<size_t>(slab, 1)));
  return (int)std::min<int64_t>({(int64_t)grid_max, groups, by_mem});
}

// shared_slab: the caller provides the lanes kernel's state (a multi launch);
// otherwise it is allocated on the DEM's device state for the pass's grid.
tmcs_status decode_prepare(const Dem& D, const tmcs_decoder_cfg& cfg, uint64_t n_shots, void* state,
                           hipStream_t stream, DecodePass* out, bool shared_slab = false) {
  DecodePass& ps = *out;
  DecodeDevice* d = (DecodeDevice*)state;
  tmcs_status st = TMCS_OK;
  if (!d && (st = ensure_device(D, &d)) != TMCS_OK) return st;
  ps.d = d;
  ps.D = &D;
  ps.cfg = cfg;
  ps.stride = (int64_t)((n_shots + 63) / 64);
  ps.full = cfg.ehat_dev || cfg.llr_dev || cfg.iters_dev || cfg.flags_dev;
  const int mw = (D.rows + 63) / 64;
  ps.mw = mw;
  int npad = OSD_THREADS;   // sort length: a power of two, at least one key per thread
  while (npad < D.cols) npad <<= 1;
  if (cfg.osd_window < 0 || cfg.osd_window > WIN_MAX_ROWS)
    return fail(TMCS_EINVAL, "osd_window must be in [0, 2048]");
  if (cfg.osd_order < 0 || cfg.osd_order > 64) return fail(TMCS_EINVAL, "osd_order must be in [0, 64]");
  if (cfg.bp_global_state < 0 || cfg.bp_global_state > 3)
    return fail(TMCS_EINVAL, "bp_global_state must be 0, 1, 2 or 3");
  if (D.cols > R_IDX || D.rows > R_IDX) return fail(TMCS_EUNSUPPORTED, "BP: more than 2^25 - 1 columns or detectors");
  // dense OSD-0 while H fits its registers and sort, windowed beyond (or on request)
  const bool osd_win = cfg.use_osd && (cfg.osd_window > 0 || npad > OSD_MAX_KEYS || mw > 32);
  if (osd_win && cfg.osd_order > 0)
    return fail(TMCS_EUNSUPPORTED, "OSD-CS needs the dense elimination (<= 2048 detectors, <= 16384 columns)");
  const int cus = device_cus();
  // BP launch shape: one team (workgroup) per shot in flight, state in LDS
  // (the packed check state needs no sign bytes, and its column slots are
  // about n: the exact size follows from the schedule; the other kernels keep the sign bytes)
  const bool pk_ok = !d->init_pk.empty() && cfg.bp_global_state <= 1;
  size_t bp_lds = (size_t)(D.rows + 1) * 16 + (size_t)D.cols * 4 + (pk_ok ? 0 : (size_t)d->E4 + 4);
  bool gstate = cfg.bp_global_state != 0 || bp_lds > 160 * 1024;
  // state in device memory: one team per shot, or on request 64 shots per
  // workgroup in the lanes of its waves (on the surface-code NL-CNOT at d = 15..29
  // that layout measured 2-5x slower than the team kernel)
  const bool lanes = gstate && cfg.bp_global_state == 2 && D.rows > 0 && D.edges > 0;
  ps.lanes = lanes;
  if (lanes) {
    const int mode = cfg.bp_sched > 0 ? cfg.bp_sched : 2;
    if ((st = get_sched(D, d, LANES_WAVES, mode, &ps.sch)) != TMCS_OK) return st;
    ps.gstate = true;
    ps.P = 64 * LANES_WAVES;
    ps.team_bytes = lanes_slab_bytes(D.rows, D.cols, d->E4);
    ps.bp_grid_max = cus * std::max(1, std::min(cfg.bp_per_cu > 0 ? cfg.bp_per_cu : 1, 2));
  }
  // (or one pass per iteration, on request)
  const bool fused = gstate && !lanes && cfg.bp_global_state == 3 && D.rows > 0;
  ps.fused = fused;
  size_t team_bytes = fused ? fused_team_bytes(D.rows, D.cols, d->E4) : (bp_lds + 255) & ~(size_t)255;
  // teams per CU: as many as fit in LDS; with the state in device memory, one
  // team of 16 waves (fewer slabs in flight: at d = 15..29 that was 1.2-1.7x
  // faster than 4 teams of 8 waves), unless the caller asks for another shape
  int team_fit = gstate ? (cfg.bp_per_cu > 0 ? 32 : 1) : std::max(1, (int)((160 * 1024) / (bp_lds + 1024)));
  int P = 64;
  if (lanes) {
  } else if (cfg.bp_threads > 0) {
    P = cfg.bp_threads;
  } else {
    // about 24 waves per CU (the passes are latency-bound: more waves, more
    // overlap), but no lane should carry much more than its share of edges
    int G = gstate ? 16 : std::max(1, std::min(16, (24 + team_fit - 1) / team_fit));
    P = 64 * G;
    const int64_t cap = std::max<int64_t>(64, (2 * D.edges / std::max(d->max_row_deg, 1)) / 64 * 64);
    while (P > 64 && P > cap) P -= 64;
  }
  P = std::min(1024, std::max(64, (P + 63) / 64 * 64));
  const int sched_mode = cfg.bp_sched > 0 ? cfg.bp_sched : 1;
  const bool pk = pk_ok && !lanes && !fused;
  if (!lanes && (st = (fused ? get_fsched : pk ? (gstate ? get_psched : get_psched_lds) : get_sched)(
                     D, d, P, sched_mode, &ps.sch)) != TMCS_OK)
    return st;
  if (pk) {
    if (!gstate) {
      bp_lds = (size_t)(ps.sch.MpkL + 1) * 16 + (size_t)(ps.sch.NpkL + 1) * 4;
      if (bp_lds > 160 * 1024) {                       // (the column slots' padding tipped it over)
        gstate = true;
        if ((st = get_psched(D, d, P, sched_mode, &ps.sch)) != TMCS_OK) return st;
      }
    }
    // device memory: check slots (plus padding and sink), column slots (plus the +BIG slot)
    if (gstate) bp_lds = (size_t)(ps.sch.Mpk4 + 2) * 16 + (size_t)(ps.sch.Npk + 1) * 4;
    team_bytes = (bp_lds + 255) & ~(size_t)255;
    team_fit = gstate ? (cfg.bp_per_cu > 0 ? 32 : 1) : std::max(1, (int)((160 * 1024) / (bp_lds + 1024)));
  }
  if (!gstate && bp_lds > 64 * 1024 && !bp_lds_allow(bp_lds)) return fail(TMCS_EUNSUPPORTED, "BP state does not fit in LDS");
  const int per_cu = std::max(1, std::min({team_fit, 32 / (P / 64), cfg.bp_per_cu > 0 ? cfg.bp_per_cu : 32}));
  ps.gstate = gstate;
  ps.pk = pk;
  ps.bp_lds = bp_lds;
  if (!lanes) {
    ps.P = P;
    ps.team_bytes = team_bytes;
    ps.bp_grid_max = cus * per_cu;
  }
  // shots per internal pass: as few passes as the OSD LLR staging allows
  // (<= 8 GiB), each ending on its slowest teams; passes of equal size
  int64_t cmax = std::max<int64_t>(DECODE_CHUNK_MIN, ((1ll << 31) / std::max(D.cols, 1)) & ~63ll);
  if (cfg.decode_chunk > 0) cmax = std::min<int64_t>(cmax, cfg.decode_chunk);
  const int64_t nch = std::max<int64_t>(1, ((int64_t)n_shots + cmax - 1) / cmax);
  const int64_t chunk = std::min<int64_t>((int64_t)n_shots, (((int64_t)n_shots + nch - 1) / nch + 63) & ~63ll);
  ps.chunk = chunk;
  // OSD launch shape
  const int W = osd_win ? 2 * WIN_MW
                        : 2 * (mw <= 1 ? 1 : mw <= 2 ? 2 : mw <= 4 ? 4 : mw <= 5 ? 5 : mw <= 8 ? 8 : mw <= 12 ? 12
                               : mw <= 15 ? 15 : mw <= 18 ? 18 : mw <= 24 ? 24 : 32);
  // rank and rows the elimination works with: H's, or a window's
  const int osd_rank = osd_win ? WIN_MAX_ROWS : D.rank;
  const int osd_rows = osd_win ? WIN_MAX_ROWS : D.rows;
  if (osd_win) npad = WIN_KEYS;
  // (+ the OSD-CS bitset of kept sorted positions after the accumulator)
  size_t osd_lds = (size_t)npad * 8 + (size_t)osd_rank * 8 + (size_t)osd_rows * 8 + (size_t)W * 8 + 64 +
                   (cfg.osd_order > 0 ? (size_t)npad / 8 + 16 : 0);
  // small DEMs keep the elimination basis in LDS as well (at least two workgroups
  // per CU); their sorted keys are stored as 32-bit column indices
  const size_t basis_bytes = (size_t)std::max(osd_rank, 1) * W * 8;
  const bool osd_bl = !osd_win && osd_lds_basis_ok(mw, npad) && osd_lds - (size_t)npad * 4 + basis_bytes <= 80 * 1024;
  if (osd_bl) osd_lds += basis_bytes - (size_t)npad * 4;
  // dense OSD-0 on a DEM wider than the prefix: prefix pass, then a full sort of the rest
  const int pfx_keys = osd_bl ? PFX_KEYS_WAVE : PFX_KEYS_WG;
  // the prefix holds at most pfx_keys - 1 columns, so at most that many pivots:
  // its basis and pivot lists need pfx_rank rows, and its grid follows from its
  // own LDS (more workgroups per CU than for the full sort; a basis in HBM is
  // sized for that grid)
  const int pfx_rank = std::min(osd_rank, pfx_keys);
  // and the one-wave variant's basis vectors carry PFX_KEYS_WAVE / 64 words of combination part
  const int W_pfx = osd_bl ? W / 2 + PFX_KEYS_WAVE / 64 : W;
  // (the one-wave variant gathers 8-byte keys over its 4-byte index area and the LDS basis after it)
  const bool osd_pfx = cfg.use_osd && !osd_win && cfg.osd_order == 0 && D.cols >= pfx_keys &&
                       (!osd_bl || (size_t)pfx_rank * W_pfx * 8 >= (size_t)pfx_keys * 4);
  size_t pfx_lds = (size_t)pfx_keys * 8 + (size_t)pfx_rank * 8 + (size_t)osd_rows * 8 + (size_t)W_pfx * 8 + 64;
  if (osd_bl) pfx_lds += (size_t)pfx_rank * W_pfx * 8 - (size_t)pfx_keys * 4;
  const int osd_fit = std::max<int>(1, (int)((160 * 1024) / (osd_lds + 512)));
  const int osd_per_cu = std::min(osd_fit, cfg.osd_per_cu > 0 ? cfg.osd_per_cu : (osd_bl ? 16 : 4));
  const int osd_grid = std::max(1, cus * osd_per_cu);
  const int pfx_fit = std::max<int>(1, (int)((160 * 1024) / (pfx_lds + 512)));
  const int pfx_grid = std::max(1, cus * std::min(pfx_fit, cfg.osd_per_cu > 0 ? cfg.osd_per_cu : 16));
  // windowed OSD-0 in two passes: a smaller window first (fewer registers and
  // less LDS, so more workgroups per compute unit, and half or a quarter of
  // the work per pivot), then the full window on the shots whose early stop
  // it does not reach.  Local rows are numbered in order of first touch in
  // both, so the smaller window's basis is a prefix of the larger's and every
  // settled shot gets the same correction.
  // The first window has WIN_SMALL_ROWS rows where the expected number of
  // detection events per shot (from the priors) is at most three quarters of
  // that, WIN_MID_ROWS where it is at most 0.9 of that, and there is none
  // beyond.  On the surface-code CNOT at p = 1e-3: d = 21 (327 events) takes
  // 512 rows (8 instead of 24 ms per 4096 shots; 1024 rows: 12 ms), d = 29
  // (about 860) 1024 rows (44 instead of 71 ms, 2 % of the shots retried; with
  // 512 rows nearly every shot outgrew the first window).  An explicit
  // osd_window always takes both passes, the first with a quarter of its rows
  // (at most WIN_SMALL_ROWS).
  const int user_rows = cfg.osd_window > 0 ? cfg.osd_window : WIN_MAX_ROWS;
  const double ev = osd_win && cfg.osd_window == 0 ? expected_events(D) : 0.0;
  const int mw1 = cfg.osd_window > 0 || ev <= 0.75 * WIN_SMALL_ROWS ? WIN_SMALL_MW : WIN_MID_MW;
  const int win1_rows = cfg.osd_window > 0 ? std::min(WIN_SMALL_ROWS, user_rows / 4) : 64 * mw1;
  const bool win2 = osd_win && win1_rows >= 2 && (cfg.osd_window > 0 || ev <= (mw1 == WIN_SMALL_MW ? 0.75 : 0.9) * win1_rows);
  const int W1 = 2 * mw1;
  const size_t win1_lds = (size_t)WIN_KEYS * 8 + (size_t)(64 * mw1) * 16 + (size_t)W1 * 8 + 64;
  const int win1_fit = std::max<int>(1, (int)((160 * 1024) / (win1_lds + 512)));
  const int win1_grid = std::max(1, cus * std::min(win1_fit, cfg.osd_per_cu > 0 ? cfg.osd_per_cu : 8));
  ps.osd_win = osd_win; ps.osd_pfx = osd_pfx; ps.osd_bl = osd_bl; ps.win2 = win2;
  ps.npad = npad; ps.pfx_keys = pfx_keys; ps.pfx_rank = pfx_rank;
  ps.osd_grid = osd_grid; ps.pfx_grid = pfx_grid; ps.osd_lds = osd_lds; ps.pfx_lds = pfx_lds;
  ps.win1_grid = win1_grid; ps.win1_lds = win1_lds; ps.win1_rows = win1_rows; ps.win1_mw = mw1;
  if ((st = grow(&d->queue, &d->cap_queue, (size_t)chunk)) != TMCS_OK) return st;
  if ((st = grow(&d->synd, &d->cap_synd, (size_t)chunk * (size_t)std::max(mw, 1))) != TMCS_OK) return st;
  if (gstate && !lanes && (st = grow(&d->gstate, &d->cap_gstate, (size_t)cus * per_cu * team_bytes)) != TMCS_OK)
    return st;
  if (lanes && !shared_slab &&
      (st = grow(&d->gstate, &d->cap_gstate, (size_t)lanes_grid(ps.bp_grid_max, ps.team_bytes, chunk) * ps.team_bytes)) !=
          TMCS_OK)
    return st;
  if (cfg.use_osd) {
    if ((st = grow(&d->osd_queue, &d->cap_osd, (size_t)chunk)) != TMCS_OK ||
        (st = grow(&d->osd_llr, &d->cap_llr, (size_t)chunk * (size_t)D.cols)) != TMCS_OK ||
        (!osd_bl && (st = grow(&d->basis, &d->cap_basis,
                               std::max({(size_t)osd_grid * (size_t)std::max(osd_rank, 1) * W,
                                         osd_pfx ? (size_t)pfx_grid * (size_t)std::max(pfx_rank, 1) * W_pfx : 0,
                                         win2 ? (size_t)win1_grid * (64 * mw1) * W1 : 0}))) != TMCS_OK))
      return st;
    if ((osd_pfx || win2) && (st = grow(&d->retry, &d->cap_retry, (size_t)chunk)) != TMCS_OK) return st;
    if (osd_win) {
      const size_t n_map = (size_t)std::max(osd_grid, win2 ? win1_grid : 0) * 2 * (size_t)std::max(D.rows, 1);
      const int32_t* before = d->rowmap;
      const size_t cap_before = d->cap_rowmap;
      if ((st = grow(&d->rowmap, &d->cap_rowmap, n_map)) != TMCS_OK) return st;
      if (d->rowmap != before || d->cap_rowmap != cap_before) {
        const int64_t g = std::min<int64_t>(((int64_t)d->cap_rowmap + 255) / 256, 4096);
        TMCS_LAUNCH("k_fill_i32", k_fill_i32, dim3((unsigned)g), dim3(256), 0, stream, d->rowmap,
                    (int64_t)d->cap_rowmap, WIN_NONE);
      }
    }
  }
  return TMCS_OK;
}

// BP kernel arguments of the chunk [s0, s0 + ns) of a pass.
BPArgs bp_args(const DecodePass& ps, const uint64_t* det_unused, uint64_t* pred, tmcs_decode_stats* stats,
               int64_t s0, int64_t ns) {
  (void)det_unused;
  const DecodeDevice* d = ps.d;
  const Dem& D = *ps.D;
  const tmcs_decoder_cfg& cfg = ps.cfg;
  BPArgs a;
  a.csched = ps.sch.c; a.vsched = ps.sch.v; a.Kc = ps.sch.Kc; a.Kv = ps.sch.Kv; a.init = d->init; a.sign0 = d->sign0;
  if (ps.gstate) {
    a.pce = ps.sch.pce; a.pve = ps.sch.pve; a.vmap = ps.sch.vmap;
    a.corig = ps.sch.corig4; a.pinit = ps.sch.pinit4; a.Mpk = ps.sch.Mpk4; a.Npk = ps.sch.Npk;
  } else {
    a.pce = ps.sch.pceL; a.pve = ps.sch.pveL; a.vmap = ps.sch.vmapL;
    a.corig = ps.sch.corigL; a.pinit = ps.sch.pinitL; a.Mpk = ps.sch.MpkL; a.Npk = ps.sch.NpkL;
  }
  a.pcs = ps.sch.pcL; a.pvs = ps.sch.pvL;
  a.pcs4 = ps.sch.pc4; a.pvs4 = ps.sch.pv4; a.lamp = ps.sch.lamp;
  a.Kc4 = ps.sch.Kc4; a.Kv4 = ps.sch.Kv4;
  a.lam = d->lam; a.obs_mask = d->obs_mask; a.ow = D.obs_words;
  a.m = D.rows; a.n = D.cols; a.E = D.edges; a.E32 = (int32_t)D.edges; a.E4 = d->E4; a.T = cfg.max_iter; a.alpha = cfg.alpha;
  a.w = cfg.weights_dev;
  a.synd = d->synd; a.mw = std::max(ps.mw, 1); a.stride = ps.stride; a.shot0 = s0; a.nshots = ns;
  a.queue = ps.full ? nullptr : d->queue;
  a.counters = d->counters; a.use_osd = cfg.use_osd; a.osd_queue = d->osd_queue; a.osd_llr = d->osd_llr;
  a.pred = pred; a.nobs = D.nobs; a.stats = stats; a.ehat = cfg.ehat_dev; a.llr = cfg.llr_dev;
  a.iters = cfg.iters_dev; a.flags = cfg.flags_dev;
  a.gstate = d->gstate; a.team_bytes = ps.team_bytes;
  a.lone = d->lone;
  for (int w = 0; w < MAX_OW; ++w) a.pm_lam[w] = d->pm_lam[w];
  a.fsched = ps.sch.f; a.Kf = ps.sch.Kf; a.csc_row = d->csc_row; a.csc_edge = d->csc_edge;
  for (int w = 0; w < MAX_OW; ++w) a.pm_iso[w] = d->pm_iso[w];
  return a;
}

// OSD kernel arguments of the chunk starting at s0.
OSDArgs osd_args(const DecodePass& ps, uint64_t* pred, tmcs_decode_stats* stats, int64_t s0) {
  const DecodeDevice* d = ps.d;
  const Dem& D = *ps.D;
  const tmcs_decoder_cfg& cfg = ps.cfg;
  OSDArgs o;
  o.col_ptr = d->col_ptr; o.csc_row = d->csc_row; o.obs_mask = d->obs_mask; o.ow = D.obs_words;
  o.m = D.rows; o.n = D.cols; o.rank = D.rank; o.synd = d->synd; o.mw = std::max(ps.mw, 1); o.stride = ps.stride;
  o.shot0 = s0;
  o.counters = d->counters; o.osd_queue = d->osd_queue; o.osd_llr = d->osd_llr; o.basis = d->basis;
  o.pred = pred; o.nobs = D.nobs; o.stats = stats; o.ehat = cfg.ehat_dev; o.flags = cfg.flags_dev;
  o.npad = ps.npad;
  o.rowmap = d->rowmap; o.win_rows = cfg.osd_window > 0 ? cfg.osd_window : WIN_MAX_ROWS;
  o.jobs = nullptr; o.cnt_total = 2; o.cnt_next = 3; o.retry = nullptr; o.order = cfg.osd_order;
  return o;
}

// Zero the predictions of a pass (all chunks).
void decode_zero_pred(const DecodePass& ps, uint64_t* pred, hipStream_t stream) {
  const int64_t total_words = (int64_t)ps.D->nobs * ps.stride;
  if (total_words) {
    const int64_t g = std::min<int64_t>((total_words + 255) / 256, 4096);
    TMCS_LAUNCH("k_zero_words", k_zero_words, dim3((unsigned)g), dim3(256), 0, stream, pred, total_words);
  }
}

// Syndrome staging of the chunk [s0, s0 + ns): counters reset, shot-major
// transpose, compaction of the non-trivial shots.
void decode_stage(const DecodePass& ps, const uint64_t* det, tmcs_decode_stats* stats, int64_t s0, int64_t ns,
                  hipStream_t stream) {
  DecodeDevice* d = ps.d;
  const Dem& D = *ps.D;
  TMCS_LAUNCH("k_zero_i32", k_zero_i32, dim3(1), dim3(64), 0, stream, d->counters, 8);
  if (stats) TMCS_LAUNCH("k_add_shots", k_add_shots, dim3(1), dim3(1), 0, stream, stats, (unsigned long long)ns);
  const int mw = ps.mw;
  {
    const int64_t nw = (ns + 63) / 64;
    const int mt = std::max(mw, 1);
    const int64_t gx = (nw + N_XCD - 1) / N_XCD * N_XCD;
    TMCS_LAUNCH("k_synd_transpose", k_synd_transpose, dim3((unsigned)gx, (unsigned)((mt + SYND_TILES - 1) / SYND_TILES)),
                dim3(64), 0, stream, det, D.rows, ps.stride, s0, ns, mt, d->synd);
  }
  if (!ps.full) {
    if (mw >= 64) {
      const int64_t g = std::min<int64_t>((ns + 3) / 4, 4096);
      TMCS_LAUNCH("k_compact", k_compact_wide, dim3((unsigned)g), dim3(256), 0, stream, d->synd, mw, ns, d->queue,
                  d->counters);
    } else {
      const int64_t g = std::min<int64_t>((ns + 256 * COMPACT_SLABS - 1) / (256 * COMPACT_SLABS), 1024);
      TMCS_LAUNCH("k_compact", k_compact, dim3((unsigned)g), dim3(256), 0, stream, d->synd, std::max(mw, 1), ns,
                  d->queue, d->counters);
    }
    if (stats) TMCS_LAUNCH("k_add_trivial", k_add_trivial, dim3(1), dim3(1), 0, stream, stats, d->counters,
                           (unsigned long long)ns);
  }
}

tmcs_status decode_bp_launch(const DecodePass& ps, const BPArgs& a, int64_t ns, hipStream_t stream) {
  const int bp_grid = (int)std::min<int64_t>((int64_t)ps.bp_grid_max, std::max<int64_t>(ns, 1));
  const BPMulti none{nullptr, 0, nullptr};
  if (ps.lanes)
    return launch_bp_lanes(a, none, ps.cfg.weights_dev != nullptr, lanes_grid(ps.bp_grid_max, ps.team_bytes, ns),
                           stream);
  if (ps.fused) return launch_bp_fused(a, none, ps.cfg.weights_dev != nullptr, bp_grid, ps.P, stream);
  launch_k_bp<false>(ps.cfg.weights_dev != nullptr, ps.gstate, ps.pk, bp_grid, ps.P, ps.gstate ? 0 : ps.bp_lds, stream,
                     a, none);
  return hip_check(hipGetLastError(), "k_bp launch");
}

tmcs_status decode_osd_launch(const DecodePass& ps, uint64_t* pred, tmcs_decode_stats* stats, int64_t s0,
                              hipStream_t stream) {
  if (!ps.cfg.use_osd) return TMCS_OK;
  const OSDArgs o = osd_args(ps, pred, stats, s0);
  if (ps.osd_win) {
    if (!ps.win2) return launch_osd_win(o, ps.osd_grid, ps.osd_lds, stream, WIN_MW);
    OSDArgs o1 = o;
    o1.retry = ps.d->retry;
    o1.win_rows = ps.win1_rows;
    tmcs_status st = launch_osd_win(o1, ps.win1_grid, ps.win1_lds, stream, ps.win1_mw);
    if (st != TMCS_OK) return st;
    OSDArgs o2 = o;
    o2.jobs = ps.d->retry; o2.cnt_total = 4; o2.cnt_next = 5;
    return launch_osd_win(o2, ps.osd_grid, ps.osd_lds, stream, WIN_MW);
  }
  if (ps.osd_pfx) {
    OSDArgs op = o;
    op.npad = ps.pfx_keys;
    op.rank = ps.pfx_rank;
    op.retry = ps.d->retry;
    tmcs_status st = dispatch_osd_pfx(ps.mw, ps.osd_bl, op, ps.pfx_grid, ps.pfx_lds, stream);
    if (st != TMCS_OK) return st;
    OSDArgs orr = o;
    orr.jobs = ps.d->retry; orr.cnt_total = 4; orr.cnt_next = 5;
    return dispatch_osd(ps.mw, ps.npad / (ps.osd_bl ? 64 : OSD_THREADS), ps.osd_bl, orr, ps.osd_grid, ps.osd_lds,
                        stream);
  }
  return dispatch_osd(ps.mw, ps.npad / (ps.osd_bl ? 64 : OSD_THREADS), ps.osd_bl, o, ps.osd_grid, ps.osd_lds, stream);
}

}  // namespace

tmcs_status decode_run(const Dem& D, const tmcs_decoder_cfg& cfg, const uint64_t* det, uint64_t n_shots,
                       uint64_t* pred, tmcs_decode_stats* stats, hipStream_t stream, void* state) {
  if (n_shots == 0) return TMCS_OK;
  if (!det && D.rows) return fail(TMCS_EINVAL, "null detector buffer");
  if (!pred && D.nobs) return fail(TMCS_EINVAL, "null prediction buffer");
  if (n_shots > (1ull << 40)) return fail(TMCS_EINVAL, "n_shots too large");
  DecodePass ps;
  tmcs_status st = decode_prepare(D, cfg, n_shots, state, stream, &ps);
  if (st != TMCS_OK) return st;
  decode_zero_pred(ps, pred, stream);
  for (int64_t s0 = 0; s0 < (int64_t)n_shots; s0 += ps.chunk) {
    const int64_t ns = std::min<int64_t>(ps.chunk, (int64_t)n_shots - s0);
    decode_stage(ps, det, stats, s0, ns, stream);
    if ((st = decode_bp_launch(ps, bp_args(ps, det, pred, stats, s0, ns), ns, stream)) != TMCS_OK) return st;
    if ((st = decode_osd_launch(ps, pred, stats, s0, stream)) != TMCS_OK) return st;
  }
  return TMCS_OK;
}

// ---------------------------------------------------------------- multi-item
// A plan's decode items run as one batch: staging per item, then one BP launch
// per group of items that share the kernel variant (state in LDS or in device
// memory) and team size, and one windowed-OSD launch for the items that use
// the windowed OSD-0 with the same grid; any other OSD runs per item, beside
// that launch on a stream of its own.
struct MultiDecode {
  struct Item {
    DecodePass ps;
    const uint64_t* det = nullptr;
    uint64_t* pred = nullptr;
    tmcs_decode_stats* stats = nullptr;
  };
  struct BPGroup {
    bool gstate = false, lanes = false, fused = false, pk = false, weighted = false;
    unsigned char* slab = nullptr;   // lanes: the state of every workgroup, shared by the group's items
    int P = 0, grid = 0;
    size_t lds = 0;
    std::vector<int> items;
    BPArgs* tab = nullptr;   // device [items]
    BPArgs first{};          // host copy of the first item's arguments
  };
  std::vector<Item> items;
  uint64_t batch = 0;
  std::vector<BPGroup> bp;
  std::vector<int> osd_win_items, osd_other_items;
  bool osd_win2 = false;     // the windowed items run the two-window scheme
  OSDArgs* osd_tab = nullptr;
  OSDArgs* osd_tab2 = nullptr;   // win2: the full window's pass over the retry lists
  OSDArgs osd_first2{};
  int osd_grid1 = 0, osd_mw1 = 0;
  size_t osd_lds1 = 0;
  OSDArgs osd_first{};       // host copy of the first windowed item's arguments
  int osd_grid = 0;
  size_t osd_lds = 0;
  int32_t* next = nullptr;   // device [2]: BP and OSD job counters of the multi launches
  // with both windowed and other OSD items: the other items' OSD runs on its own
  // stream beside the windowed launch (forked from and joined back to the
  // caller's stream by events; branches of a captured graph)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

void decode_multi_free(MultiDecode* m) {
  if (!m) return;
  for (auto& g : m->bp) { hipFree(g.tab); hipFree(g.slab); }
  hipFree(m->osd_tab);
  hipFree(m->osd_tab2);
  hipFree(m->next);
  if (m->side) (void)hipStreamDestroy(m->side);
  if (m->fork) (void)hipEventDestroy(m->fork);
  if (m->join) (void)hipEventDestroy(m->join);
  delete m;
}

tmcs_status decode_multi_create(const std::vector<MultiItemSpec>& specs, uint64_t batch, hipStream_t stream,
                                MultiDecode** out) {
  *out = nullptr;
  if (specs.empty() || specs.size() > (size_t)MAX_MULTI) return fail(TMCS_EINVAL, "multi decode: 1..16 items");
  MultiDecode* m = new MultiDecode();
  m->batch = batch;
  tmcs_status st = TMCS_OK;
  for (const auto& sp : specs) {
    MultiDecode::Item it;
    it.det = sp.det; it.pred = sp.pred; it.stats = sp.stats;
    if (sp.cfg.ehat_dev || sp.cfg.llr_dev || sp.cfg.iters_dev || sp.cfg.flags_dev) st = fail(TMCS_EINVAL, "multi decode: no per-shot outputs");
    if (st == TMCS_OK) st = decode_prepare(*sp.D, sp.cfg, batch, sp.state, stream, &it.ps, true);
    if (st == TMCS_OK && it.ps.chunk < (int64_t)batch) st = fail(TMCS_EUNSUPPORTED, "multi decode: batch exceeds one decoder pass");
    if (st != TMCS_OK) { decode_multi_free(m); return st; }
    m->items.push_back(it);
  }
  // BP groups: (state placement, team size)
  for (int i = 0; i < (int)m->items.size(); ++i) {
    const DecodePass& ps = m->items[i].ps;
    MultiDecode::BPGroup* g = nullptr;
    for (auto& q : m->bp)
      if (q.gstate == ps.gstate && q.lanes == ps.lanes && q.fused == ps.fused && q.pk == ps.pk && q.P == ps.P) g = &q;
    if (!g) {
      m->bp.push_back(MultiDecode::BPGroup());
      g = &m->bp.back();
      g->gstate = ps.gstate;
      g->lanes = ps.lanes;
      g->fused = ps.fused;
      g->pk = ps.pk;
      g->P = ps.P;
      g->grid = ps.bp_grid_max;
    }
    g->items.push_back(i);
    g->weighted = g->weighted || ps.cfg.weights_dev != nullptr;
    g->grid = std::min(g->grid, ps.bp_grid_max);
    if (!ps.gstate) g->lds = std::max(g->lds, ps.bp_lds);
  }
  // Heaviest items first in every group (workgroups take the items in order):
  // the launch then ends on the cheapest shots instead of waiting for the last
  // teams of the largest DEM.  Weight: edges, then the expected detection events
  // (at one DEM size, more events mean more BP iterations).
  {
    std::vector<double> ev(m->items.size());
    for (size_t i = 0; i < m->items.size(); ++i) ev[i] = expected_events(*m->items[i].ps.D);
    for (auto& g : m->bp)
      std::stable_sort(g.items.begin(), g.items.end(), [&](int x, int y) {
        const int64_t ex = m->items[x].ps.D->edges, ey = m->items[y].ps.D->edges;
        return ex != ey ? ex > ey : ev[x] > ev[y];
      });
  }
  const int cus = device_cus();
  for (auto& g : m->bp) {
    if (!g.gstate) {
      // teams resident per CU with the largest state of the group
      const int fit = std::max(1, std::min((int)((160 * 1024) / (g.lds + 1024)), 32 / (g.P / 64)));
      g.grid = std::min(g.grid, cus * fit);
      if (g.lds > 64 * 1024 && !bp_lds_allow(g.lds)) {
        decode_multi_free(m);
        return fail(TMCS_EUNSUPPORTED, "BP state does not fit in LDS");
      }
    }
    if (g.lanes) {
      // one state slab per workgroup sized for the largest item
      size_t slab = 0;
      for (int i : g.items) slab = std::max(slab, m->items[i].ps.team_bytes);
      g.lds = slab;
      g.grid = lanes_grid(g.grid, slab, (int64_t)batch * (int64_t)g.items.size());
      if (hipMalloc((void**)&g.slab, (size_t)g.grid * slab) != hipSuccess) {
        decode_multi_free(m);
        return fail(TMCS_ENOMEM, "hipMalloc failed (BP state of the multi decode)");
      }
    }
    std::vector<BPArgs> tab;
    for (int i : g.items) {
      const auto& it = m->items[i];
      tab.push_back(bp_args(it.ps, it.det, it.pred, it.stats, 0, (int64_t)batch));
      if (g.lanes) {
        tab.back().gstate = g.slab;
        tab.back().team_bytes = g.lds;
      }
    }
    g.first = tab[0];
    if ((st = upload(&g.tab, tab)) != TMCS_OK) { decode_multi_free(m); return st; }
  }
  // windowed OSD: one launch for the items sharing its grid and LDS
  for (int i = 0; i < (int)m->items.size(); ++i) {
    const DecodePass& ps = m->items[i].ps;
    if (!ps.cfg.use_osd) continue;
    const bool join = ps.osd_win && (m->osd_win_items.empty() || (ps.osd_grid == m->osd_grid && ps.osd_lds == m->osd_lds &&
                                                               ps.win2 == m->osd_win2 && ps.win1_grid == m->osd_grid1 &&
                                                               ps.win1_lds == m->osd_lds1 && ps.win1_mw == m->osd_mw1));
    if (join) {
      m->osd_win_items.push_back(i);
      m->osd_grid = ps.osd_grid;
      m->osd_lds = ps.osd_lds;
      m->osd_win2 = ps.win2;
      m->osd_grid1 = ps.win1_grid;
      m->osd_lds1 = ps.win1_lds;
      m->osd_mw1 = ps.win1_mw;
    } else {
      m->osd_other_items.push_back(i);
    }
  }
  if (!m->osd_win_items.empty()) {
    std::vector<OSDArgs> tab;
    std::vector<OSDArgs> tab2;
    for (int i : m->osd_win_items) {
      const DecodePass& ps = m->items[i].ps;
      OSDArgs o = osd_args(ps, m->items[i].pred, m->items[i].stats, 0);
      if (m->osd_win2) {
        OSDArgs o2 = o;
        o2.jobs = ps.d->retry; o2.cnt_total = 4; o2.cnt_next = 5;
        tab2.push_back(o2);
        o.retry = ps.d->retry;
        o.win_rows = ps.win1_rows;
      }
      tab.push_back(o);
    }
    m->osd_first = tab[0];
    if ((st = upload(&m->osd_tab, tab)) != TMCS_OK) { decode_multi_free(m); return st; }
    if (m->osd_win2) {
      m->osd_first2 = tab2[0];
      if ((st = upload(&m->osd_tab2, tab2)) != TMCS_OK) { decode_multi_free(m); return st; }
    }
  }
  if (hipMalloc((void**)&m->next, 3 * sizeof(int32_t)) != hipSuccess) {
    decode_multi_free(m);
    return fail(TMCS_ENOMEM, "hipMalloc failed (multi decode counters)");
  }
  if (!m->osd_win_items.empty() && !m->osd_other_items.empty()) {
    st = hip_check(hipStreamCreate(&m->side), "hipStreamCreate");
    if (st == TMCS_OK) st = hip_check(hipEventCreateWithFlags(&m->fork, hipEventDisableTiming), "hipEventCreate");
    if (st == TMCS_OK) st = hip_check(hipEventCreateWithFlags(&m->join, hipEventDisableTiming), "hipEventCreate");
    if (st != TMCS_OK) { decode_multi_free(m); return st; }
  }
  *out = m;
  return TMCS_OK;
}

// One batch of every item: staging, the grouped BP launches, the OSD launches.
tmcs_status decode_multi_enqueue(MultiDecode* m, hipStream_t stream) {
  const int64_t ns = (int64_t)m->batch;
  for (auto& it : m->items) {
    decode_zero_pred(it.ps, it.pred, stream);
    decode_stage(it.ps, it.det, it.stats, 0, ns, stream);
  }
  TMCS_LAUNCH("k_zero_i32", k_zero_i32, dim3(1), dim3(64), 0, stream, m->next, 3);
  tmcs_status st;
  for (auto& g : m->bp) {
    // (the BP job counter is shared by the groups in turn: zeroed before each)
    if (&g != &m->bp.front()) TMCS_LAUNCH("k_zero_i32", k_zero_i32, dim3(1), dim3(64), 0, stream, m->next, 1);
    const BPMulti mu{g.tab, (int32_t)g.items.size(), m->next};
    const int grid = std::max(1, g.grid);
    const BPArgs& a0 = g.first;
    if (g.lanes) {
      if ((st = launch_bp_lanes(a0, mu, g.weighted, grid, stream)) != TMCS_OK) return st;
      continue;
    }
    if (g.fused) {
      if ((st = launch_bp_fused(a0, mu, g.weighted, grid, g.P, stream)) != TMCS_OK) return st;
      continue;
    }
    launch_k_bp<true>(g.weighted, g.gstate, g.pk, grid, g.P, g.gstate ? 0 : g.lds, stream, a0, mu);
    if ((st = hip_check(hipGetLastError(), "k_bp launch")) != TMCS_OK) return st;
  }
  // Items outside the windowed launch (another window shape, or no window) take
  // their OSD on the side stream when there is one: the two chains then share
  // the GPU, and each one's full-window retries (a few shots, one workgroup each,
  // bound by a workgroup's latency) run while the other still fills it.
  if (m->side) {
    if ((st = hip_check(hipEventRecord(m->fork, stream), "multi decode fork")) != TMCS_OK) return st;
    if ((st = hip_check(hipStreamWaitEvent(m->side, m->fork, 0), "multi decode fork wait")) != TMCS_OK) return st;
    for (int i : m->osd_other_items) {
      auto& it = m->items[i];
      if ((st = decode_osd_launch(it.ps, it.pred, it.stats, 0, m->side)) != TMCS_OK) return st;
    }
    if ((st = hip_check(hipEventRecord(m->join, m->side), "multi decode join")) != TMCS_OK) return st;
  }
  if (!m->osd_win_items.empty()) {
    const OSDMulti mu{m->osd_tab, (int32_t)m->osd_win_items.size(), m->next + 1};
    if (m->osd_win2) {
      if ((st = launch_osd_win_multi(m->osd_first, mu, m->osd_grid1, m->osd_lds1, stream, m->osd_mw1)) != TMCS_OK)
        return st;
      const OSDMulti mu2{m->osd_tab2, (int32_t)m->osd_win_items.size(), m->next + 2};
      if ((st = launch_osd_win_multi(m->osd_first2, mu2, m->osd_grid, m->osd_lds, stream, WIN_MW)) != TMCS_OK) return st;
    } else if ((st = launch_osd_win_multi(m->osd_first, mu, m->osd_grid, m->osd_lds, stream, WIN_MW)) != TMCS_OK) {
      return st;
    }
  }
  if (m->side) return hip_check(hipStreamWaitEvent(stream, m->join, 0), "multi decode join wait");
  for (int i : m->osd_other_items) {
    auto& it = m->items[i];
    if ((st = decode_osd_launch(it.ps, it.pred, it.stats, 0, stream)) != TMCS_OK) return st;
  }
  return TMCS_OK;
}

__global__ void k_count_errors(const uint64_t* __restrict__ pred, const uint64_t* __restrict__ obs, uint32_t k,
                               int64_t stride, uint64_t n_shots, unsigned long long* out) {
  unsigned long long local = 0;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < stride; w += (int64_t)gridDim.x * blockDim.x) {
    uint64_t x = 0;
    for (uint32_t o = 0; o < k; ++o) x |= pred[(int64_t)o * stride + w] ^ obs[(int64_t)o * stride + w];
    const uint64_t left = n_shots - (uint64_t)w * 64;
    if (left < 64) x &= (1ull << left) - 1ull;
    local += (unsigned long long)__popcll(x);
  }
  if (local) atomicAdd(out, local);
}

// One error counter per device, allocated on the first call there and reused;
// the lock is held until the count has been read back, so calls never share it.
std::mutex g_ler_mu;
unsigned long long* g_ler_count[64] = {};

tmcs_status ler_run(const uint64_t* pred, const uint64_t* obs, uint32_t k, uint64_t n_shots, uint64_t* n_err,
                    hipStream_t stream) {
  *n_err = 0;
  if (n_shots == 0 || k == 0) return TMCS_OK;
  if (!pred || !obs) return fail(TMCS_EINVAL, "null buffer");
  int dev = 0;
  tmcs_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st != TMCS_OK) return st;
  if (dev < 0 || dev >= 64) return fail(TMCS_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_ler_mu);
  if (!g_ler_count[dev] &&
      (st = hip_check(hipMalloc((void**)&g_ler_count[dev], sizeof(unsigned long long)), "hipMalloc")) != TMCS_OK)
    return st;
  unsigned long long* dcount = g_ler_count[dev];
  TMCS_LAUNCH("k_zero_words", k_zero_words, dim3(1), dim3(64), 0, stream, (uint64_t*)dcount, (int64_t)1);
  const int64_t stride = (int64_t)((n_shots + 63) / 64);
  const int64_t g = std::min<int64_t>((stride + 255) / 256, 2048);
  TMCS_LAUNCH("k_count_errors", k_count_errors, dim3((unsigned)g), dim3(256), 0, stream, pred, obs, k, stride, n_shots, dcount);
  unsigned long long h = 0;
  st = hip_check(hipMemcpyAsync(&h, dcount, sizeof(h), hipMemcpyDeviceToHost, stream), "copy error count");
  if (st == TMCS_OK) st = hip_check(hipStreamSynchronize(stream), "ler synchronize");
  if (st != TMCS_OK) return st;
  *n_err = h;
  return TMCS_OK;
}

tmcs_status count_errors_async(const uint64_t* pred, const uint64_t* obs, uint32_t k, uint64_t n_shots,
                               unsigned long long* counter, hipStream_t stream) {
  if (n_shots == 0 || k == 0) return TMCS_OK;
  const int64_t stride = (int64_t)((n_shots + 63) / 64);
  const int64_t g = std::min<int64_t>((stride + 255) / 256, 2048);
  TMCS_LAUNCH("k_count_errors", k_count_errors, dim3((unsigned)g), dim3(256), 0, stream, pred, obs, k, stride, n_shots,
              counter);
  return hip_check(hipGetLastError(), "k_count_errors launch");
}

// Launch-shape search: decode the caller's syndromes with every candidate shape
// and keep the fastest.  Results never depend on the launch shape, only time.
// The autotuner's choices, cached per (GPU, DEM shape, decoder settings):
// a later call with the same key returns the cached launch fields at once.
struct TuneKey {
  std::string arch;
  int rows, cols, rank, obs;
  int64_t edges;
  int max_iter, use_osd, osd_order, osd_window, weighted, global_state;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, rows, cols, rank, obs, edges, max_iter, use_osd, osd_order, osd_window, weighted, global_state) <
           std::tie(o.arch, o.rows, o.cols, o.rank, o.obs, o.edges, o.max_iter, o.use_osd, o.osd_order, o.osd_window,
                    o.weighted, o.global_state);
  }
};
struct TuneVal { int bp_threads, bp_per_cu, osd_per_cu, bp_sched; };
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;

tmcs_status autotune_run(const Dem& D, const uint64_t* det, uint64_t n_shots, tmcs_decoder_cfg* cfg,
                         hipStream_t stream) {
  if (n_shots == 0) return fail(TMCS_EINVAL, "autotune needs shots");
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(TMCS_EDEVICE, "no HIP device");
  const TuneKey key{std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount), D.rows, D.cols,
                    D.rank, D.nobs, D.edges, cfg->max_iter, cfg->use_osd, cfg->osd_order, cfg->osd_window,
                    cfg->weights_dev != nullptr, cfg->bp_global_state};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      cfg->bp_threads = it->second.bp_threads;
      cfg->bp_per_cu = it->second.bp_per_cu;
      cfg->osd_per_cu = it->second.osd_per_cu;
      cfg->bp_sched = it->second.bp_sched;
      return TMCS_OK;
    }
  }
  uint64_t* pred = nullptr;
  const int64_t stride = (int64_t)((n_shots + 63) / 64);
  if (hipMalloc((void**)&pred, (size_t)std::max(D.nobs, 1) * stride * 8) != hipSuccess)
    return fail(TMCS_ENOMEM, "hipMalloc (autotune)");
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  tmcs_decoder_cfg base = *cfg;
  base.ehat_dev = nullptr; base.llr_dev = nullptr; base.iters_dev = nullptr; base.flags_dev = nullptr;
  tmcs_decoder_cfg best = base;
  float best_ms = 1e30f;
  const int threads[] = {64, 128, 256, 512, 1024};
  const int bp_cu[] = {0, 4};
  const int osd_cu[] = {2, 4, 8};
  const int sched[] = {1, 2};
  tmcs_status st = TMCS_OK;
  for (int th : threads)
    for (int bc : bp_cu)
      for (int oc : osd_cu)
        for (int sm : sched) {
        tmcs_decoder_cfg c = base;
        c.bp_threads = th; c.bp_per_cu = bc; c.osd_per_cu = oc; c.bp_sched = sm;
        if ((st = decode_run(D, c, det, n_shots, pred, nullptr, stream)) != TMCS_OK) break;   // warm
        (void)hipEventRecord(e0, stream);
        if ((st = decode_run(D, c, det, n_shots, pred, nullptr, stream)) != TMCS_OK) break;
        (void)hipEventRecord(e1, stream);
        if ((st = hip_check(hipEventSynchronize(e1), "autotune")) != TMCS_OK) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) { best_ms = ms; best = c; }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  hipFree(pred);
  if (st != TMCS_OK) return st;
  cfg->bp_threads = best.bp_threads;
  cfg->bp_per_cu = best.bp_per_cu;
  cfg->osd_per_cu = best.osd_per_cu;
  cfg->bp_sched = best.bp_sched;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[key] = TuneVal{best.bp_threads, best.bp_per_cu, best.osd_per_cu, best.bp_sched};
  return TMCS_OK;
}

void* decode_state_new(const Dem& D, tmcs_status* st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { *st = fail(TMCS_EDEVICE, "no HIP device"); return nullptr; }
  DecodeDevice* d = nullptr;
  *st = build_state(D, dev, &d);
  return d;
}

void decode_state_free(void* state) {
  DecodeDevice* d = (DecodeDevice*)state;
  if (!d) return;
  free_device(d);
  delete d;
}

void decode_release(Dem& D) {
  DecodeDevice* d = (DecodeDevice*)D.device;
  if (!d) return;
  free_device(d);
  delete d;
  D.device = nullptr;
}

}  // namespace tmcs
