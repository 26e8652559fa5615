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
// registers, then among themselves in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "../host/device.h"
#include "../host/timing.h"

namespace tmcs {

namespace {

constexpr float BP_BIG = 1e30f;
constexpr int OSD_THREADS = 256;
constexpr int OSD_MAX_KEYS = 16384;

struct DecodeDevice {
  int device = -1;
  int32_t *row_ptr = nullptr, *col_idx = nullptr, *col_ptr = nullptr, *csc_row = nullptr, *csc_edge = nullptr;
  float* lam = nullptr;
  uint64_t* obs_mask = nullptr;
  // scratch
  int32_t* counters = nullptr;     // [0] queue len, [1] bp next, [2] osd len, [3] osd next
  int32_t* queue = nullptr;
  int32_t* osd_queue = nullptr;
  float* osd_llr = nullptr;
  uint64_t* basis = nullptr;
  uint64_t* synd = nullptr;
  size_t cap_queue = 0, cap_osd = 0, cap_llr = 0, cap_basis = 0, cap_synd = 0;
};

struct BPArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* col_ptr;
  const int32_t* csc_row;
  const int32_t* csc_edge;
  const float* lam;
  const uint64_t* obs_mask;
  int32_t m, n;
  int64_t E;
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
};

__device__ __forceinline__ void write_pred(uint64_t* pred, int64_t stride, int nobs, int64_t shot, uint64_t mask) {
  for (int o = 0; o < nobs; ++o)
    if ((mask >> o) & 1ull)
      atomicOr((unsigned long long*)&pred[(int64_t)o * stride + (shot >> 6)], (unsigned long long)(1ull << (shot & 63)));
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

__global__ void k_zero_words(uint64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_add_shots(tmcs_decode_stats* stats, unsigned long long n) {
  if (threadIdx.x == 0) atomicAdd((unsigned long long*)&stats->shots, n);
}

__global__ void k_zero_i32(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Detector-major bit planes -> shot-major syndrome words for the chunk
// [shot0, shot0 + nshots): one workgroup per (64-shot word, 64-detector tile),
// a 64 x 64 bit transpose through LDS.
__global__ void __launch_bounds__(64) k_synd_transpose(const uint64_t* __restrict__ det, int32_t m, int64_t stride,
                                                       int64_t shot0, int64_t nshots, int32_t mw,
                                                       uint64_t* __restrict__ synd) {
  __shared__ uint64_t tile[64];
  const int lane = threadIdx.x;
  const int64_t w = blockIdx.x;             // shot word within the chunk
  const int rt = blockIdx.y;                // detector tile
  const int row = rt * 64 + lane;
  tile[lane] = row < m ? det[(int64_t)row * stride + (shot0 >> 6) + w] : 0ull;
  __syncthreads();
  uint64_t out = 0ull;
#pragma unroll 16
  for (int i = 0; i < 64; ++i) out |= ((tile[i] >> lane) & 1ull) << i;
  const int64_t s = w * 64 + lane;
  if (s < nshots) synd[s * mw + rt] = out;
}

// Queue the shots of the chunk whose syndrome is non-zero.
__global__ void k_compact(const uint64_t* __restrict__ synd, int32_t mw, int64_t nshots,
                          int32_t* __restrict__ queue, int32_t* __restrict__ counters) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nshots; s += (int64_t)gridDim.x * blockDim.x) {
    uint64_t any = 0ull;
    for (int k = 0; k < mw; ++k) any |= synd[s * mw + k];
    if (any) queue[atomicAdd(&counters[0], 1)] = (int32_t)s;
  }
}

// Slot states of the BP kernel.
enum : int32_t { SLOT_EMPTY = 0, SLOT_NEW = 1, SLOT_ACTIVE = 2, SLOT_DONE = 3 };

// BP over a persistent workgroup that carries S shots ("slots") at once, each at
// its own iteration; a slot whose shot has converged (or used its T iterations)
// is finalised and refilled from the queue independently of the others.
//
// MSG = true keeps every check-to-variable message m_{c->v} in LDS (CSR edge
// order); the check pass first turns m_old into q = L_v - m_old in place, then
// writes the new messages, and the variable pass is a plain sum.  MSG = false
// keeps the compressed check state instead - (min1, min2, argmin edge, sign
// parity) per check and one sign bit per edge - and rebuilds messages from it;
// it needs ~4 bytes per column + 13 per check instead of 4 per edge, for DEMs
// whose messages do not fit.
template <bool MSG>
__global__ void k_bp(BPArgs a, int32_t S) {
  extern __shared__ __align__(8) unsigned char sm[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = a.m, n = a.n;
  const int64_t E = a.E;
  const int64_t nwords = (E + 31) / 32;
  // per-slot arrays (slot-major)
  float* Lf = (float*)sm;                                             // [S][n]
  float* msg = Lf + (size_t)S * n;                                    // MSG:  [S][E]
  float* min1 = msg;                                                  // !MSG: [S][m]
  float* min2 = min1 + (size_t)S * m;                                 // !MSG: [S][m]
  int32_t* arg = (int32_t*)(min2 + (size_t)S * m);                    // !MSG: [S][m]
  uint32_t* esign = (uint32_t*)(arg + (size_t)S * m);                 // !MSG: [S][nwords]
  uint8_t* cflag = MSG ? (uint8_t*)(msg + (size_t)S * E) : (uint8_t*)(esign + (size_t)S * nwords);  // [S][m]
  __shared__ int32_t st[16], tt[16], ls_of[16], flag[16], osdpos[16], itr[16];
  __shared__ unsigned long long pmask[16];
  __shared__ int s_exit;
  const int32_t total = a.queue ? a.counters[0] : (int32_t)a.nshots;
  if (tid < S) {
    const int job = atomicAdd(&a.counters[1], 1);
    st[tid] = job < total ? SLOT_NEW : SLOT_EMPTY;
    ls_of[tid] = job < total ? (a.queue ? a.queue[job] : job) : 0;
    flag[tid] = 0;
  }
  __syncthreads();
  while (true) {
    // 1. initialise new slots: syndrome bits, zero messages / check state, L = lambda
    for (int sl = 0; sl < S; ++sl) {
      if (st[sl] != SLOT_NEW) continue;
      const uint64_t* sy = a.synd + (int64_t)ls_of[sl] * a.mw;
      uint8_t* cf = cflag + sl * m;
      for (int c = tid; c < m; c += nt) {
        const int sb = (int)((sy[c >> 6] >> (c & 63)) & 1ull);
        cf[c] = (uint8_t)(sb << 1);
        if (!MSG) {
          min1[sl * m + c] = 0.0f;
          min2[sl * m + c] = 0.0f;
          arg[sl * m + c] = -1;
        }
        if (sb) flag[sl] = 1;                              // benign race: every writer stores 1
      }
      float* L = Lf + (size_t)sl * n;
      for (int v = tid; v < n; v += nt) L[v] = a.lam[v];
      if (MSG) {
        float* ms = msg + (size_t)sl * E;
        for (int64_t e = tid; e < E; e += nt) ms[e] = 0.0f;
      } else {
        uint32_t* es = esign + (size_t)sl * nwords;
        for (int64_t i = tid; i < nwords; i += nt) es[i] = 0u;
      }
    }
    __syncthreads();
    if (tid < S && st[tid] == SLOT_NEW) {
      if (flag[tid]) { st[tid] = SLOT_ACTIVE; tt[tid] = 1; flag[tid] = 0; }
      else { st[tid] = SLOT_DONE; itr[tid] = 0; osdpos[tid] = -1; flag[tid] = 1; pmask[tid] = 0ull; }
    }
    __syncthreads();
    // 2. check pass: convergence of L^{(t-1)} and the messages of iteration t
    for (int sl = 0; sl < S; ++sl) {
      if (st[sl] != SLOT_ACTIVE) continue;
      const int t = tt[sl];
      const bool update = t <= a.T;
      const float* L = Lf + (size_t)sl * n;
      const uint8_t* cf = cflag + sl * m;
      int unsat = 0;
      for (int c = tid; c < m; c += nt) {
        const int32_t r0 = a.row_ptr[c], r1 = a.row_ptr[c + 1];
        const int sc = (cf[c] >> 1) & 1;
        int hard = 0, npar = 0;
        float n1 = BP_BIG, n2 = BP_BIG;
        int32_t nag = -1;
        if (MSG) {
          float* ms = msg + (size_t)sl * E;
          for (int32_t e = r0; e < r1; ++e) {
            const float Lv = L[a.col_idx[e]];
            hard ^= Lv < 0.0f ? 1 : 0;
            const float q = __fsub_rn(Lv, ms[e]);           // q_{v->c} = L_v - m_old
            ms[e] = q;
            const float aq = fabsf(q);
            if (aq < n1) { n2 = n1; n1 = aq; nag = e; }
            else if (aq < n2) { n2 = aq; }
            npar ^= q < 0.0f ? 1 : 0;
          }
          if (update) {
            const float* wt = a.w ? a.w + (int64_t)(t - 1) * E : nullptr;
            for (int32_t e = r0; e < r1; ++e) {
              const float q = ms[e];
              const float at = wt ? wt[e] : a.alpha;
              const float mag = __fmul_rn(at, e == nag ? n2 : n1);
              ms[e] = (sc ^ npar ^ (q < 0.0f ? 1 : 0)) ? -mag : mag;
            }
          }
        } else {
          uint32_t* es = esign + (size_t)sl * nwords;
          const float m1 = min1[sl * m + c], m2 = min2[sl * m + c];
          const int32_t ag = arg[sl * m + c];
          const int sp = cf[c] & 1;
          for (int32_t e0 = r0; e0 < r1; e0 += 4) {
            int32_t vv[4];
            float Lv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) vv[u] = e0 + u < r1 ? a.col_idx[e0 + u] : 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) Lv[u] = L[vv[u]];
            const int32_t elast = e0 + 3 < r1 ? e0 + 3 : r1 - 1;   // a batch spans <= 2 sign words
            const uint32_t sw0 = es[e0 >> 5], sw1 = es[elast >> 5];
            uint32_t flip0 = 0u, flip1 = 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int32_t e = e0 + u;
              if (e >= r1) break;
              hard ^= Lv[u] < 0.0f ? 1 : 0;
              if (!update) continue;
              const bool hi = (e >> 5) != (e0 >> 5);
              const int se = (int)(((hi ? sw1 : sw0) >> (e & 31)) & 1u);
              const float aold = (t == 1) ? 1.0f : (a.w ? a.w[(int64_t)(t - 2) * E + e] : a.alpha);
              const float mag = __fmul_rn(aold, e == ag ? m2 : m1);
              const float mo = (sc ^ sp ^ se) ? -mag : mag;
              const float q = __fsub_rn(Lv[u], mo);
              const float aq = fabsf(q);
              const int ng = q < 0.0f ? 1 : 0;
              if (aq < n1) { n2 = n1; n1 = aq; nag = e; }
              else if (aq < n2) { n2 = aq; }
              npar ^= ng;
              if (ng != se) {
                if (hi) flip1 |= 1u << (e & 31); else flip0 |= 1u << (e & 31);
              }
            }
            if (flip0) atomicXor(&es[e0 >> 5], flip0);
            if (flip1) atomicXor(&es[elast >> 5], flip1);
          }
          if (update) {
            min1[sl * m + c] = n1;
            min2[sl * m + c] = n2;
            arg[sl * m + c] = nag;
            cflag[sl * m + c] = (uint8_t)((sc << 1) | npar);
          }
        }
        unsat |= hard != sc;
      }
      if (unsat) flag[sl] = 1;                               // benign race: every writer stores 1
    }
    __syncthreads();
    // 3. per-slot decision: converged, out of iterations, or one more iteration
    if (tid < S && st[tid] == SLOT_ACTIVE) {
      const int t = tt[tid];
      const bool conv = flag[tid] == 0;
      if (conv || t > a.T) {
        st[tid] = SLOT_DONE;
        itr[tid] = conv ? t - 1 : a.T;
        flag[tid] = conv ? 1 : 0;                           // flag now = converged
        pmask[tid] = 0ull;
        osdpos[tid] = (!conv && a.use_osd) ? atomicAdd(&a.counters[2], 1) : -1;
      } else {
        flag[tid] = 0;
      }
    }
    __syncthreads();
    // 4. variable pass for active slots, finalisation for finished ones
    for (int sl = 0; sl < S; ++sl) {
      const int state = st[sl];
      float* L = Lf + (size_t)sl * n;
      if (state == SLOT_ACTIVE) {
        if (MSG) {
          const float* ms = msg + (size_t)sl * E;
          for (int v = tid; v < n; v += nt) {
            float acc = a.lam[v];
            const int32_t k0 = a.col_ptr[v], k1 = a.col_ptr[v + 1];
            for (int32_t k = k0; k < k1; ++k) acc = __fadd_rn(acc, ms[a.csc_edge[k]]);
            L[v] = acc;
          }
        } else {
          const int t = tt[sl];
          const uint32_t* es = esign + (size_t)sl * nwords;
          for (int v = tid; v < n; v += nt) {
            float acc = a.lam[v];
            const int32_t k0 = a.col_ptr[v], k1 = a.col_ptr[v + 1];
            for (int32_t k = k0; k < k1; ++k) {
              const int32_t c = sl * m + a.csc_row[k], e = a.csc_edge[k];
              const uint8_t fl = cflag[c];
              const int se = (int)((es[e >> 5] >> (e & 31)) & 1u);
              const float at = a.w ? a.w[(int64_t)(t - 1) * E + e] : a.alpha;
              const float mag = __fmul_rn(at, e == arg[c] ? min2[c] : min1[c]);
              const int neg = ((fl >> 1) ^ fl ^ se) & 1;
              acc = __fadd_rn(acc, neg ? -mag : mag);
            }
            L[v] = acc;
          }
        }
      } else if (state == SLOT_DONE) {
        const int64_t shot = a.shot0 + ls_of[sl];
        const int pos = osdpos[sl];
        for (int v = tid; v < n; v += nt) {
          const float Lv = L[v];
          if (pos < 0 && Lv < 0.0f && a.obs_mask[v]) atomicXor(&pmask[sl], (unsigned long long)a.obs_mask[v]);
          if (pos >= 0) a.osd_llr[(int64_t)pos * n + v] = Lv;
          if (a.llr) a.llr[shot * n + v] = Lv;
          if (a.ehat && pos < 0) a.ehat[shot * n + v] = Lv < 0.0f ? 1 : 0;
        }
      }
    }
    __syncthreads();
    // 5. finished slots: predictions, statistics, refill
    if (tid < S) {
      if (st[tid] == SLOT_ACTIVE) {
        tt[tid] += 1;
      } else if (st[tid] == SLOT_DONE) {
        const int64_t shot = a.shot0 + ls_of[tid];
        const bool conv = flag[tid] != 0;
        const int pos = osdpos[tid];
        if (pos < 0) write_pred(a.pred, a.stride, a.nobs, shot, pmask[tid]);
        else a.osd_queue[pos] = ls_of[tid];
        if (a.iters) a.iters[shot] = itr[tid];
        if (a.flags) a.flags[shot] = (uint8_t)((conv ? 1 : 0) | (pos >= 0 ? 2 : 0));
        if (a.stats) {
          if (itr[tid] > 0 || !conv) atomicAdd((unsigned long long*)&a.stats->nontrivial, 1ull);
          if (conv) atomicAdd((unsigned long long*)&a.stats->converged, 1ull);
          if (pos >= 0) atomicAdd((unsigned long long*)&a.stats->osd, 1ull);
          atomicAdd((unsigned long long*)&a.stats->bp_iters, (unsigned long long)itr[tid]);
        }
        const int job = atomicAdd(&a.counters[1], 1);
        st[tid] = job < total ? SLOT_NEW : SLOT_EMPTY;
        ls_of[tid] = job < total ? (a.queue ? a.queue[job] : job) : 0;
        flag[tid] = 0;
      }
    }
    if (tid == 0) s_exit = 1;
    __syncthreads();
    if (tid < S && st[tid] != SLOT_EMPTY) s_exit = 0;     // benign race: every writer stores 0
    __syncthreads();
    if (s_exit) break;
  }
}

// ------------------------------------------------------------------ OSD-0
struct OSDArgs {
  const int32_t* col_ptr;
  const int32_t* csc_row;
  const uint64_t* obs_mask;
  int32_t m, n, rank;
  const uint64_t* det;
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
  int32_t npad;              // sort length (power of two >= n)
};

__device__ __forceinline__ uint32_t order_key(float x) {
  if (x == 0.0f) x = 0.0f;   // -0 and +0 compare equal
  const uint32_t b = __float_as_uint(x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Wave-uniform broadcast of lane `src`'s 64-bit value (src must be wave-uniform).
__device__ __forceinline__ uint64_t bcast64(uint64_t x, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of npad = OSD_THREADS * KPT 64-bit keys, ascending.  Thread t
// holds elements t*KPT .. t*KPT+KPT-1 in registers; partners within a thread are
// compared in registers, partners within a wave via lane shuffles, and only the
// strides that cross waves go through LDS (`keys`), which also receives the
// sorted result.
template <int KPT>
__device__ __forceinline__ void bitonic_sort_regs(uint64_t (&x)[KPT], uint64_t* keys, int npad) {
  const int tid = threadIdx.x;
  for (int k = 2; k <= npad; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < KPT) {
#pragma unroll
        for (int jj = KPT / 2; jj >= 1; jj >>= 1) {
          if (jj != j) continue;
#pragma unroll
          for (int r = 0; r < KPT; ++r) {
            if (r & jj) continue;
            const int e = tid * KPT + r;
            const bool up = (e & k) == 0;
            const uint64_t a0 = x[r], a1 = x[r | jj];
            const bool sw = (a0 > a1) == up;
            x[r] = sw ? a1 : a0;
            x[r | jj] = sw ? a0 : a1;
          }
        }
      } else if (j < KPT * 64) {
        const int tj = j / KPT;                       // partner lane distance
        const bool lower = (tid & tj) == 0;
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
          const int e = tid * KPT + r;
          const bool up = (e & k) == 0;
          const uint64_t y = __shfl_xor(x[r], tj, 64);
          // the lower element of the pair keeps the minimum when sorting up
          const bool take_min = lower == up;
          x[r] = take_min ? (x[r] < y ? x[r] : y) : (x[r] > y ? x[r] : y);
        }
      } else {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < KPT; ++r) keys[tid * KPT + r] = x[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
          const int e = tid * KPT + r;
          const bool up = (e & k) == 0;
          const uint64_t y = keys[e ^ j];
          const bool take_min = ((e & j) == 0) == up;
          x[r] = take_min ? (x[r] < y ? x[r] : y) : (x[r] > y ? x[r] : y);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < KPT; ++r) keys[tid * KPT + r] = x[r];
  __syncthreads();
}

// Bit p of a register-resident bit vector (p < 64 * MW).
template <int MW, int W>
__device__ __forceinline__ uint64_t bit_of(const uint64_t (&v)[W], int p) {
  uint64_t pw = 0ull;
#pragma unroll
  for (int w = 0; w < MW; ++w)
    if ((p >> 6) == w) pw = v[w];
  return (pw >> (p & 63)) & 1ull;
}

// W = words per basis vector: MW syndrome words then RW combination words.
//
// The basis is kept fully reduced: basis vector i has a 1 at its pivot row p_i
// and 0 at every other pivot row.  A candidate column h is then reduced by
// XORing exactly the basis vectors whose pivot rows lie in supp(h) (at most the
// column degree), and a syndrome s by those whose pivot rows lie in supp(s).
// New basis vectors are created 64 at a time by one wave, made fully reduced
// among themselves, and the older vectors are then reduced against them.
template <int MW, int RW, int KPT>
__global__ void __launch_bounds__(OSD_THREADS) k_osd(OSDArgs a) {
  constexpr int W = MW + RW;
  extern __shared__ __align__(8) unsigned char sm[];
  uint64_t* keys = (uint64_t*)sm;                                  // [npad]
  int32_t* pivot = (int32_t*)(keys + a.npad);                      // [rank] pivot row of basis i
  int32_t* kept = pivot + a.rank;                                  // [rank] column of basis i
  int32_t* prow = kept + a.rank;                                   // [m] basis index of a pivot row, or -1
  uint64_t* acc = (uint64_t*)(((uintptr_t)(prow + a.m) + 7) & ~(uintptr_t)7);  // [W] solve accumulator
  __shared__ int s_job, s_r;
  __shared__ uint64_t s_red;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  uint64_t* B = a.basis + (int64_t)blockIdx.x * a.rank * W;
  while (true) {
    if (tid == 0) s_job = atomicAdd(&a.counters[3], 1);
    __syncthreads();
    const int job = s_job;
    __syncthreads();
    if (job >= a.counters[2]) break;
    const int64_t ls = a.osd_queue[job];
    const int64_t shot = a.shot0 + ls;
    const float* L = a.osd_llr + (int64_t)job * a.n;
    // 1. sort columns by (L_v, v)
    for (int r = tid; r < a.m; r += OSD_THREADS) prow[r] = -1;
    if (tid < W) acc[tid] = 0ull;
    if (tid == 0) s_r = 0;
    {
      uint64_t x[KPT];
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        const int i = tid * KPT + r;
        x[r] = i < a.n ? (((uint64_t)order_key(L[i]) << 32) | (uint32_t)i) : ~0ull;
      }
      bitonic_sort_regs<KPT>(x, keys, a.npad);
    }
    // 2. information set, 256 sorted candidates per pass (one per thread)
    for (int base = 0; base < a.n; base += OSD_THREADS) {
      const int r_start = s_r;
      __syncthreads();           // every wave has read s_r before wave 0 advances it
      if (r_start >= a.rank) break;
      const int idx = base + tid;
      const int col = idx < a.n ? (int)(keys[idx] & 0xFFFFFFFFu) : -1;
      uint64_t v[W];
#pragma unroll
      for (int w = 0; w < W; ++w) v[w] = 0ull;
      if (col >= 0) {
        const int32_t k0 = a.col_ptr[col], k1 = a.col_ptr[col + 1];
        for (int32_t k = k0; k < k1; ++k) {
          const int r = a.csc_row[k];
#pragma unroll
          for (int w = 0; w < MW; ++w)
            if ((r >> 6) == w) v[w] ^= 1ull << (r & 63);
        }
        // phase 1: the basis vectors pivoted on rows of h
        for (int32_t k = k0; k < k1; ++k) {
          const int i = prow[a.csc_row[k]];
          if (i >= 0) {
            const uint64_t* b = B + (int64_t)i * W;
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] ^= b[w];
          }
        }
      }
      __syncthreads();           // phase 1 everywhere before any wave publishes new pivots
      int r_done = r_start;
      for (int q = 0; q < OSD_THREADS / 64; ++q) {
        if (wave == q) {
          // phase 2: in-order pass over this wave's candidates whose syndrome
          // part is still nonzero (zero ones depend on earlier columns)
          int r = r_done;
          int mine = -1;      // pivot row of the basis vector this lane became
          auto nz = [&]() {
            uint64_t o = 0ull;
#pragma unroll
            for (int w = 0; w < MW; ++w) o |= v[w];
            return o != 0ull && col >= 0;
          };
          uint64_t live = __ballot(nz());
          while (live && r < a.rank) {
            const int j = __ffsll((unsigned long long)live) - 1;
            uint64_t b[W];
#pragma unroll
            for (int w = 0; w < W; ++w) b[w] = bcast64(v[w], j);
            int p = -1;
#pragma unroll
            for (int w = 0; w < MW; ++w)
              if (p < 0 && b[w]) p = w * 64 + (__ffsll((unsigned long long)b[w]) - 1);
#pragma unroll
            for (int w = 0; w < RW; ++w)
              if (w == (r >> 6)) b[MW + w] ^= 1ull << (r & 63);   // the column itself
            if (lane == j) {
#pragma unroll
              for (int w = 0; w < W; ++w) v[w] = b[w];
              mine = p;
              pivot[r] = p;
              kept[r] = col;
              prow[p] = r;
            }
            const uint64_t mask = (lane > j) ? 0ull - bit_of<MW, W>(v, p) : 0ull;
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] ^= b[w] & mask;
            ++r;
            live = __ballot(lane > j && nz());
          }
          // make the new vectors fully reduced among themselves (latest first)
          uint64_t piv_lanes = __ballot(mine >= 0);
          while (piv_lanes) {
            const int j = 63 - __clzll((long long)piv_lanes);
            piv_lanes &= ~(1ull << j);
            const int pj = __builtin_amdgcn_readlane(mine, j);
            uint64_t b[W];
#pragma unroll
            for (int w = 0; w < W; ++w) b[w] = bcast64(v[w], j);
            const uint64_t mask = (mine >= 0 && lane < j) ? 0ull - bit_of<MW, W>(v, pj) : 0ull;
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] ^= b[w] & mask;
          }
          if (mine >= 0) {
            const int i = prow[mine];
#pragma unroll
            for (int w = 0; w < W; ++w) B[(int64_t)i * W + w] = v[w];
          }
          if (lane == 0) s_r = r;
        }
        __syncthreads();
        const int r_new = s_r;
        if (r_new > r_done) {
          // older basis vectors: clear their bits at the new pivots
          for (int i = tid; i < r_done; i += OSD_THREADS) {
            uint64_t bi[W];
#pragma unroll
            for (int w = 0; w < W; ++w) bi[w] = B[(int64_t)i * W + w];
            bool changed = false;
            for (int j = r_done; j < r_new; ++j) {
              if (bit_of<MW, W>(bi, pivot[j])) {
                const uint64_t* bj = B + (int64_t)j * W;
#pragma unroll
                for (int w = 0; w < W; ++w) bi[w] ^= bj[w];
                changed = true;
              }
            }
            if (changed) {
#pragma unroll
              for (int w = 0; w < W; ++w) B[(int64_t)i * W + w] = bi[w];
            }
          }
          // candidates of later waves: reduce against the new vectors
          if (wave > q) {
            uint64_t m[W];
#pragma unroll
            for (int w = 0; w < W; ++w) m[w] = 0ull;
            for (int j = r_done; j < r_new; ++j) {
              const uint64_t msk = 0ull - bit_of<MW, W>(v, pivot[j]);
              const uint64_t* bj = B + (int64_t)j * W;
#pragma unroll
              for (int w = 0; w < W; ++w) m[w] ^= bj[w] & msk;
            }
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] ^= m[w];
          }
        }
        r_done = r_new;
        __syncthreads();
      }
    }
    // 3. solve: s reduced by the basis vectors pivoted on rows of s
    const int r = s_r;
    int bad = 0;
    for (int row = tid; row < a.m; row += OSD_THREADS) {
      if ((a.det[(int64_t)row * a.stride + (shot >> 6)] >> (shot & 63)) & 1ull) {
        atomicXor((unsigned long long*)&acc[row >> 6], (unsigned long long)(1ull << (row & 63)));
        const int i = prow[row];
        if (i >= 0) {
          const uint64_t* b = B + (int64_t)i * W;
#pragma unroll
          for (int w = 0; w < W; ++w)
            if (b[w]) atomicXor((unsigned long long*)&acc[w], (unsigned long long)b[w]);
        }
      }
    }
    __syncthreads();
    for (int w = tid; w < MW; w += OSD_THREADS) bad |= acc[w] != 0ull;
    const int not_in_span = __syncthreads_or(bad);
    uint64_t pm = 0;
    if (a.ehat)
      for (int v = tid; v < a.n; v += OSD_THREADS) a.ehat[shot * a.n + v] = 0;
    __syncthreads();
    for (int i = tid; i < r; i += OSD_THREADS) {
      if ((acc[MW + (i >> 6)] >> (i & 63)) & 1ull) {
        const int col = kept[i];
        pm ^= a.obs_mask[col];
        if (a.ehat) a.ehat[shot * a.n + col] = 1;
      }
    }
    pm = block_xor_u64(pm, &s_red);
    if (tid == 0) {
      write_pred(a.pred, a.stride, a.nobs, shot, pm);
      if (a.flags) a.flags[shot] = (uint8_t)(2 | (not_in_span ? 4 : 0));
      if (a.stats && not_in_span) atomicAdd((unsigned long long*)&a.stats->not_in_span, 1ull);
    }
    __syncthreads();
  }
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
  hipFree(d->osd_llr); hipFree(d->basis); hipFree(d->synd);
  *d = DecodeDevice();
}

tmcs_status build_state(const Dem& D, int dev, DecodeDevice** out) {
  DecodeDevice* d = new DecodeDevice();
  d->device = dev;
  std::vector<int32_t> csc_row(D.row_idx.begin(), D.row_idx.end());
  std::vector<float> lam(D.cols);
  for (int j = 0; j < D.cols; ++j) lam[j] = (float)std::log((1.0 - D.priors[j]) / D.priors[j]);
  tmcs_status st;
  if ((st = upload(&d->row_ptr, D.row_ptr)) != TMCS_OK || (st = upload(&d->col_idx, D.col_idx)) != TMCS_OK ||
      (st = upload(&d->col_ptr, D.col_ptr)) != TMCS_OK || (st = upload(&d->csc_row, csc_row)) != TMCS_OK ||
      (st = upload(&d->csc_edge, D.csc_edge)) != TMCS_OK || (st = upload(&d->lam, lam)) != TMCS_OK ||
      (st = upload(&d->obs_mask, D.obs_mask)) != TMCS_OK) {
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

template <int MW, int RW, int KPT>
tmcs_status launch_osd(const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_osd<MW, RW, KPT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return fail(TMCS_EUNSUPPORTED, "OSD workspace does not fit in LDS");
  TMCS_LAUNCH("k_osd", (k_osd<MW, RW, KPT>), dim3(grid), dim3(OSD_THREADS), lds, s, a);
  return hip_check(hipGetLastError(), "k_osd launch");
}

template <int MW>
tmcs_status dispatch_kpt(int kpt, const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (kpt) {
    case 1: return launch_osd<MW, MW, 1>(a, grid, lds, s);
    case 2: return launch_osd<MW, MW, 2>(a, grid, lds, s);
    case 4: return launch_osd<MW, MW, 4>(a, grid, lds, s);
    case 8: return launch_osd<MW, MW, 8>(a, grid, lds, s);
    case 16: return launch_osd<MW, MW, 16>(a, grid, lds, s);
    case 32: return launch_osd<MW, MW, 32>(a, grid, lds, s);
    case 64: return launch_osd<MW, MW, 64>(a, grid, lds, s);
    default: return fail(TMCS_EUNSUPPORTED, "OSD sort size");
  }
}

tmcs_status dispatch_osd(int mw, int kpt, const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  if (mw <= 1) return dispatch_kpt<1>(kpt, a, grid, lds, s);
  if (mw <= 2) return dispatch_kpt<2>(kpt, a, grid, lds, s);
  if (mw <= 4) return dispatch_kpt<4>(kpt, a, grid, lds, s);
  if (mw <= 5) return dispatch_kpt<5>(kpt, a, grid, lds, s);
  if (mw <= 8) return dispatch_kpt<8>(kpt, a, grid, lds, s);
  if (mw <= 12) return dispatch_kpt<12>(kpt, a, grid, lds, s);
  if (mw <= 15) return dispatch_kpt<15>(kpt, a, grid, lds, s);
  if (mw <= 18) return dispatch_kpt<18>(kpt, a, grid, lds, s);
  if (mw <= 24) return dispatch_kpt<24>(kpt, a, grid, lds, s);
  if (mw <= 32) return dispatch_kpt<32>(kpt, a, grid, lds, s);
  return fail(TMCS_EUNSUPPORTED, "OSD supports at most 2048 detectors in this build");
}

constexpr int64_t DECODE_CHUNK_MIN = 4096;

}  // namespace

tmcs_status decode_run(const Dem& D, const tmcs_decoder_cfg& cfg, const uint64_t* det, uint64_t n_shots,
                       uint64_t* pred, tmcs_decode_stats* stats, hipStream_t stream, void* state) {
  if (n_shots == 0) return TMCS_OK;
  if (!det && D.rows) return fail(TMCS_EINVAL, "null detector buffer");
  if (!pred && D.nobs) return fail(TMCS_EINVAL, "null prediction buffer");
  if (n_shots > (1ull << 40)) return fail(TMCS_EINVAL, "n_shots too large");
  DecodeDevice* d = (DecodeDevice*)state;
  tmcs_status st = TMCS_OK;
  if (!d && (st = ensure_device(D, &d)) != TMCS_OK) return st;
  const int64_t stride = (int64_t)((n_shots + 63) / 64);
  const bool full = cfg.ehat_dev || cfg.llr_dev || cfg.iters_dev || cfg.flags_dev;
  const int mw = (D.rows + 63) / 64;
  int npad = OSD_THREADS;   // sort length: a power of two, at least one key per thread
  while (npad < D.cols) npad <<= 1;
  if (cfg.use_osd && (npad > OSD_MAX_KEYS || mw > 32))
    return fail(TMCS_EUNSUPPORTED, "OSD-0 supports up to 16384 columns and 2048 detectors in this build");
  const int cus = device_cus();
  // BP launch shape: explicit messages when they fit, S shots per workgroup
  int bp_threads = cfg.bp_threads > 0 ? cfg.bp_threads : (D.cols > 4096 ? 512 : 256);
  bp_threads = std::min(1024, std::max(64, (bp_threads + 63) / 64 * 64));
  const size_t per_shot_msg = (size_t)D.cols * 4 + (size_t)D.edges * 4 + (size_t)D.rows;
  const size_t per_shot_cmp = (size_t)D.cols * 4 + (size_t)D.rows * 13 + (size_t)((D.edges + 31) / 32) * 4;
  const bool use_msg = per_shot_msg + 16 <= 64 * 1024;
  const size_t per_shot = use_msg ? per_shot_msg : per_shot_cmp;
  if (per_shot + 16 > 160 * 1024) return fail(TMCS_EUNSUPPORTED, "BP state exceeds the 160 KB LDS of one workgroup");
  int slots = cfg.bp_slots > 0 ? cfg.bp_slots : 1;
  slots = std::max(1, std::min(16, slots));
  while (slots > 1 && per_shot * slots + 16 > 160 * 1024) --slots;
  const size_t bp_lds = per_shot * slots + 16;
  const void* bp_fn = use_msg ? (const void*)k_bp<true> : (const void*)k_bp<false>;
  if (bp_lds > 64 * 1024 &&
      hipFuncSetAttribute(bp_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bp_lds) != hipSuccess)
    return fail(TMCS_EUNSUPPORTED, "BP state does not fit in LDS");
  const int per_cu_fit = std::max<int>(1, (int)((160 * 1024) / (bp_lds + 512)));
  const int per_cu = std::min(per_cu_fit, cfg.bp_per_cu > 0 ? cfg.bp_per_cu : 16);
  // shots per internal pass: bounded so the OSD LLR staging stays <= 1 GiB
  const int64_t chunk = std::min<int64_t>((int64_t)n_shots,
                                          std::max<int64_t>(DECODE_CHUNK_MIN, ((1ll << 28) / std::max(D.cols, 1)) & ~63ll));
  // OSD launch shape
  const int W = 2 * (mw <= 1 ? 1 : mw <= 2 ? 2 : mw <= 4 ? 4 : mw <= 5 ? 5 : mw <= 8 ? 8 : mw <= 12 ? 12
                   : mw <= 15 ? 15 : mw <= 18 ? 18 : mw <= 24 ? 24 : 32);
  const size_t osd_lds = (size_t)npad * 8 + (size_t)D.rank * 8 + (size_t)D.rows * 4 + (size_t)W * 8 + 64;
  const int osd_fit = std::max<int>(1, (int)((160 * 1024) / (osd_lds + 512)));
  const int osd_per_cu = std::min(osd_fit, cfg.osd_per_cu > 0 ? cfg.osd_per_cu : 4);
  const int osd_grid = std::max(1, cus * osd_per_cu);
  if ((st = grow(&d->queue, &d->cap_queue, (size_t)chunk)) != TMCS_OK) return st;
  if ((st = grow(&d->synd, &d->cap_synd, (size_t)chunk * (size_t)std::max(mw, 1))) != TMCS_OK) return st;
  if (cfg.use_osd) {
    if ((st = grow(&d->osd_queue, &d->cap_osd, (size_t)chunk)) != TMCS_OK ||
        (st = grow(&d->osd_llr, &d->cap_llr, (size_t)chunk * (size_t)D.cols)) != TMCS_OK ||
        (st = grow(&d->basis, &d->cap_basis, (size_t)osd_grid * (size_t)std::max(D.rank, 1) * W)) != TMCS_OK)
      return st;
  }
  const int64_t total_words = (int64_t)D.nobs * stride;
  if (total_words) {
    const int64_t g = std::min<int64_t>((total_words + 255) / 256, 4096);
    TMCS_LAUNCH("k_zero_words", k_zero_words, dim3((unsigned)g), dim3(256), 0, stream, pred, total_words);
  }
  for (int64_t s0 = 0; s0 < (int64_t)n_shots; s0 += chunk) {
    const int64_t ns = std::min<int64_t>(chunk, (int64_t)n_shots - s0);
    TMCS_LAUNCH("k_zero_i32", k_zero_i32, dim3(1), dim3(64), 0, stream, d->counters, 8);
    if (stats) TMCS_LAUNCH("k_add_shots", k_add_shots, dim3(1), dim3(1), 0, stream, stats, (unsigned long long)ns);
    {
      const int64_t nw = (ns + 63) / 64;
      const int mt = std::max(mw, 1);
      TMCS_LAUNCH("k_synd_transpose", k_synd_transpose, dim3((unsigned)nw, (unsigned)mt), dim3(64), 0, stream, det,
                  D.rows, stride, s0, ns, mt, d->synd);
    }
    if (!full) {
      const int64_t g = std::min<int64_t>((ns + 255) / 256, 4096);
      TMCS_LAUNCH("k_compact", k_compact, dim3((unsigned)g), dim3(256), 0, stream, d->synd, std::max(mw, 1), ns,
                  d->queue, d->counters);
    }
    BPArgs a;
    a.row_ptr = d->row_ptr; a.col_idx = d->col_idx; a.col_ptr = d->col_ptr; a.csc_row = d->csc_row;
    a.csc_edge = d->csc_edge; a.lam = d->lam; a.obs_mask = d->obs_mask;
    a.m = D.rows; a.n = D.cols; a.E = D.edges; a.T = cfg.max_iter; a.alpha = cfg.alpha; a.w = cfg.weights_dev;
    a.synd = d->synd; a.mw = std::max(mw, 1); a.stride = stride; a.shot0 = s0; a.nshots = ns; a.queue = full ? nullptr : d->queue;
    a.counters = d->counters; a.use_osd = cfg.use_osd; a.osd_queue = d->osd_queue; a.osd_llr = d->osd_llr;
    a.pred = pred; a.nobs = D.nobs; a.stats = stats; a.ehat = cfg.ehat_dev; a.llr = cfg.llr_dev;
    a.iters = cfg.iters_dev; a.flags = cfg.flags_dev;
    const int bp_grid = (int)std::min<int64_t>((int64_t)cus * per_cu, std::max<int64_t>((ns + slots - 1) / slots, 1));
    if (use_msg)
      TMCS_LAUNCH("k_bp", k_bp<true>, dim3(bp_grid), dim3(bp_threads), bp_lds, stream, a, (int32_t)slots);
    else
      TMCS_LAUNCH("k_bp", k_bp<false>, dim3(bp_grid), dim3(bp_threads), bp_lds, stream, a, (int32_t)slots);
    if ((st = hip_check(hipGetLastError(), "k_bp launch")) != TMCS_OK) return st;
    if (cfg.use_osd) {
      OSDArgs o;
      o.col_ptr = d->col_ptr; o.csc_row = d->csc_row; o.obs_mask = d->obs_mask;
      o.m = D.rows; o.n = D.cols; o.rank = D.rank; o.det = det; o.stride = stride; o.shot0 = s0;
      o.counters = d->counters; o.osd_queue = d->osd_queue; o.osd_llr = d->osd_llr; o.basis = d->basis;
      o.pred = pred; o.nobs = D.nobs; o.stats = stats; o.ehat = cfg.ehat_dev; o.flags = cfg.flags_dev;
      o.npad = npad;
      if ((st = dispatch_osd(mw, npad / OSD_THREADS, o, osd_grid, osd_lds, stream)) != TMCS_OK) return st;
    }
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

tmcs_status ler_run(const uint64_t* pred, const uint64_t* obs, uint32_t k, uint64_t n_shots, uint64_t* n_err,
                    hipStream_t stream) {
  *n_err = 0;
  if (n_shots == 0 || k == 0) return TMCS_OK;
  if (!pred || !obs) return fail(TMCS_EINVAL, "null buffer");
  unsigned long long* dcount = nullptr;
  tmcs_status st = hip_check(hipMalloc((void**)&dcount, sizeof(unsigned long long)), "hipMalloc");
  if (st != TMCS_OK) return st;
  TMCS_LAUNCH("k_zero_words", k_zero_words, dim3(1), dim3(64), 0, stream, (uint64_t*)dcount, (int64_t)1);
  const int64_t stride = (int64_t)((n_shots + 63) / 64);
  const int64_t g = std::min<int64_t>((stride + 255) / 256, 2048);
  TMCS_LAUNCH("k_count_errors", k_count_errors, dim3((unsigned)g), dim3(256), 0, stream, pred, obs, k, stride, n_shots, dcount);
  unsigned long long h = 0;
  st = hip_check(hipMemcpyAsync(&h, dcount, sizeof(h), hipMemcpyDeviceToHost, stream), "copy error count");
  if (st == TMCS_OK) st = hip_check(hipStreamSynchronize(stream), "ler synchronize");
  hipFree(dcount);
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
tmcs_status autotune_run(const Dem& D, const uint64_t* det, uint64_t n_shots, tmcs_decoder_cfg* cfg,
                         hipStream_t stream) {
  if (n_shots == 0) return fail(TMCS_EINVAL, "autotune needs shots");
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
  const int threads[] = {128, 256, 512};
  const int bp_cu[] = {4, 16};
  const int osd_cu[] = {2, 4, 8};
  tmcs_status st = TMCS_OK;
  for (int th : threads)
    for (int bc : bp_cu)
      for (int oc : osd_cu) {
        tmcs_decoder_cfg c = base;
        c.bp_threads = th; c.bp_per_cu = bc; c.osd_per_cu = oc; c.bp_slots = 1;
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
  cfg->bp_slots = best.bp_slots;
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
