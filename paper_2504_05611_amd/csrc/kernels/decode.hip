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
  size_t cap_queue = 0, cap_osd = 0, cap_llr = 0, cap_basis = 0;
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
  const uint64_t* det;       // [m][stride]
  int64_t stride;
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

// Queue the shots of [shot0, shot0 + nshots) whose syndrome is non-zero.
__global__ void k_compact(const uint64_t* __restrict__ det, int32_t m, int64_t stride, int64_t shot0,
                          int64_t nshots, int32_t* __restrict__ queue, int32_t* __restrict__ counters,
                          tmcs_decode_stats* stats) {
  const int64_t nw = (nshots + 63) / 64;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gw = (shot0 >> 6) + w;   // shot0 is a multiple of 64
    uint64_t any = 0;
    for (int r = 0; r < m; ++r) any |= det[(int64_t)r * stride + gw];
    const int64_t left = nshots - w * 64;
    if (left < 64) any &= (1ull << left) - 1ull;
    const int cnt = __popcll(any);
    if (cnt) {
      int pos = atomicAdd(&counters[0], cnt);
      while (any) {
        const int b = __ffsll((unsigned long long)any) - 1;
        any &= any - 1;
        queue[pos++] = (int32_t)(w * 64 + b);
      }
    }
  }
}

__global__ void k_bp(BPArgs a) {
  extern __shared__ __align__(8) unsigned char sm[];
  float* Lf = (float*)sm;
  float* min1 = Lf + a.n;
  float* min2 = min1 + a.m;
  int32_t* arg = (int32_t*)(min2 + a.m);
  uint32_t* esign = (uint32_t*)(arg + a.m);
  uint8_t* cflag = (uint8_t*)(esign + (a.E + 31) / 32);
  __shared__ int s_job;
  __shared__ uint64_t s_red;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int32_t total = a.queue ? a.counters[0] : (int32_t)a.nshots;
  while (true) {
    if (tid == 0) s_job = atomicAdd(&a.counters[1], 1);
    __syncthreads();
    const int job = s_job;
    __syncthreads();
    if (job >= total) break;
    const int64_t ls = a.queue ? a.queue[job] : job;   // shot within the chunk
    const int64_t shot = a.shot0 + ls;                  // shot within the call
    int has = 0;
    for (int c = tid; c < a.m; c += nt) {
      const int s = (int)((a.det[(int64_t)c * a.stride + (shot >> 6)] >> (shot & 63)) & 1ull);
      has |= s;
      cflag[c] = (uint8_t)(s << 1);
      min1[c] = 0.0f;
      min2[c] = 0.0f;
      arg[c] = -1;
    }
    for (int v = tid; v < a.n; v += nt) Lf[v] = a.lam[v];
    for (int64_t i = tid; i < (a.E + 31) / 32; i += nt) esign[i] = 0u;
    const int nonzero = __syncthreads_or(has);
    int iters = 0;
    bool conv = !nonzero;
    if (nonzero) {
      for (int t = 1; t <= a.T + 1; ++t) {
        // check pass: convergence of L^{(t-1)}, then new check state from q^{(t-1)}
        const bool update = t <= a.T;
        int unsat = 0;
        for (int c = tid; c < a.m; c += nt) {
          const int32_t r0 = a.row_ptr[c], r1 = a.row_ptr[c + 1];
          const float m1 = min1[c], m2 = min2[c];
          const int32_t ag = arg[c];
          const uint8_t fl = cflag[c];
          const int sc = (fl >> 1) & 1, sp = fl & 1;
          int hard = 0, npar = 0;
          float n1 = BP_BIG, n2 = BP_BIG;
          int32_t nag = -1;
          for (int32_t e = r0; e < r1; ++e) {
            const int32_t v = a.col_idx[e];
            const float Lv = Lf[v];
            hard ^= Lv < 0.0f ? 1 : 0;
            if (!update) continue;
            const int se = (int)((esign[e >> 5] >> (e & 31)) & 1u);
            const float aold = (t == 1) ? 1.0f : (a.w ? a.w[(int64_t)(t - 2) * a.E + e] : a.alpha);
            const float mag = __fmul_rn(aold, e == ag ? m2 : m1);
            const float mo = (sc ^ sp ^ se) ? -mag : mag;
            const float q = __fsub_rn(Lv, mo);
            const float aq = fabsf(q);
            const int ng = q < 0.0f ? 1 : 0;
            if (aq < n1) { n2 = n1; n1 = aq; nag = e; }
            else if (aq < n2) { n2 = aq; }
            npar ^= ng;
            if (ng != se) atomicXor(&esign[e >> 5], 1u << (e & 31));
          }
          unsat |= hard != sc;
          if (update) {
            min1[c] = n1;
            min2[c] = n2;
            arg[c] = nag;
            cflag[c] = (uint8_t)((sc << 1) | npar);
          }
        }
        const int any_unsat = __syncthreads_or(unsat);
        if (!any_unsat) { conv = true; iters = t - 1; break; }
        if (!update) { iters = a.T; break; }
        // variable pass
        for (int v = tid; v < a.n; v += nt) {
          float acc = a.lam[v];
          const int32_t k0 = a.col_ptr[v], k1 = a.col_ptr[v + 1];
          for (int32_t k = k0; k < k1; ++k) {
            const int32_t c = a.csc_row[k], e = a.csc_edge[k];
            const uint8_t fl = cflag[c];
            const int se = (int)((esign[e >> 5] >> (e & 31)) & 1u);
            const float at = a.w ? a.w[(int64_t)(t - 1) * a.E + e] : a.alpha;
            const float mag = __fmul_rn(at, e == arg[c] ? min2[c] : min1[c]);
            const int neg = ((fl >> 1) ^ fl ^ se) & 1;
            acc = __fadd_rn(acc, neg ? -mag : mag);
          }
          Lf[v] = acc;
        }
        __syncthreads();
      }
    }
    // outputs
    const bool to_osd = !conv && a.use_osd;
    int osd_pos = 0;
    if (to_osd) {
      if (tid == 0) s_job = atomicAdd(&a.counters[2], 1);
      __syncthreads();
      osd_pos = s_job;
      __syncthreads();
    }
    uint64_t pm = 0;
    for (int v = tid; v < a.n; v += nt) {
      const float L = Lf[v];
      if (!to_osd && L < 0.0f) pm ^= a.obs_mask[v];
      if (to_osd) a.osd_llr[(int64_t)osd_pos * a.n + v] = L;
      if (a.llr) a.llr[shot * a.n + v] = L;
      if (a.ehat && !to_osd) a.ehat[shot * a.n + v] = L < 0.0f ? 1 : 0;
    }
    if (!to_osd) {
      pm = block_xor_u64(pm, &s_red);
      if (tid == 0) write_pred(a.pred, a.stride, a.nobs, shot, pm);
    } else if (tid == 0) {
      a.osd_queue[osd_pos] = (int32_t)ls;
    }
    if (tid == 0) {
      if (a.iters) a.iters[shot] = iters;
      if (a.flags) a.flags[shot] = (uint8_t)((conv ? 1 : 0) | (to_osd ? 2 : 0));
      if (a.stats) {
        if (nonzero) atomicAdd((unsigned long long*)&a.stats->nontrivial, 1ull);
        if (conv) atomicAdd((unsigned long long*)&a.stats->converged, 1ull);
        if (to_osd) atomicAdd((unsigned long long*)&a.stats->osd, 1ull);
        atomicAdd((unsigned long long*)&a.stats->bp_iters, (unsigned long long)iters);
      }
    }
    __syncthreads();
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
  hipFree(d->osd_llr); hipFree(d->basis);
  *d = DecodeDevice();
}

tmcs_status ensure_device(const Dem& dc, DecodeDevice** out) {
  Dem& D = const_cast<Dem&>(dc);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TMCS_EDEVICE, "no HIP device");
  DecodeDevice* d = (DecodeDevice*)D.device;
  if (d && d->device == dev) { *out = d; return TMCS_OK; }
  if (d) { free_device(d); delete d; D.device = nullptr; }
  d = new DecodeDevice();
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
                       uint64_t* pred, tmcs_decode_stats* stats, hipStream_t stream) {
  if (n_shots == 0) return TMCS_OK;
  if (!det && D.rows) return fail(TMCS_EINVAL, "null detector buffer");
  if (!pred && D.nobs) return fail(TMCS_EINVAL, "null prediction buffer");
  if (n_shots > (1ull << 40)) return fail(TMCS_EINVAL, "n_shots too large");
  DecodeDevice* d = nullptr;
  tmcs_status st = ensure_device(D, &d);
  if (st != TMCS_OK) return st;
  const int64_t stride = (int64_t)((n_shots + 63) / 64);
  const bool full = cfg.ehat_dev || cfg.llr_dev || cfg.iters_dev || cfg.flags_dev;
  const int mw = (D.rows + 63) / 64;
  int npad = OSD_THREADS;   // sort length: a power of two, at least one key per thread
  while (npad < D.cols) npad <<= 1;
  if (cfg.use_osd && (npad > OSD_MAX_KEYS || mw > 32))
    return fail(TMCS_EUNSUPPORTED, "OSD-0 supports up to 16384 columns and 2048 detectors in this build");
  const int cus = device_cus();
  // BP launch shape
  int bp_threads = cfg.bp_threads > 0 ? cfg.bp_threads : (D.cols > 4096 ? 256 : (D.cols > 512 ? 128 : 64));
  bp_threads = std::min(1024, std::max(64, (bp_threads + 63) / 64 * 64));
  const size_t bp_lds = (size_t)D.cols * 4 + (size_t)D.rows * 12 + (size_t)((D.edges + 31) / 32) * 4 +
                        (size_t)D.rows + 16;
  if (bp_lds > 160 * 1024) return fail(TMCS_EUNSUPPORTED, "BP state exceeds the 160 KB LDS of one workgroup");
  if (bp_lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_bp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bp_lds) != hipSuccess)
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
    if (!full) {
      const int64_t nw = (ns + 63) / 64;
      const int64_t g = std::min<int64_t>((nw + 255) / 256, 4096);
      TMCS_LAUNCH("k_compact", k_compact, dim3((unsigned)g), dim3(256), 0, stream, det, D.rows, stride, s0, ns,
                         d->queue, d->counters, stats);
    }
    BPArgs a;
    a.row_ptr = d->row_ptr; a.col_idx = d->col_idx; a.col_ptr = d->col_ptr; a.csc_row = d->csc_row;
    a.csc_edge = d->csc_edge; a.lam = d->lam; a.obs_mask = d->obs_mask;
    a.m = D.rows; a.n = D.cols; a.E = D.edges; a.T = cfg.max_iter; a.alpha = cfg.alpha; a.w = cfg.weights_dev;
    a.det = det; a.stride = stride; a.shot0 = s0; a.nshots = ns; a.queue = full ? nullptr : d->queue;
    a.counters = d->counters; a.use_osd = cfg.use_osd; a.osd_queue = d->osd_queue; a.osd_llr = d->osd_llr;
    a.pred = pred; a.nobs = D.nobs; a.stats = stats; a.ehat = cfg.ehat_dev; a.llr = cfg.llr_dev;
    a.iters = cfg.iters_dev; a.flags = cfg.flags_dev;
    const int bp_grid = (int)std::min<int64_t>((int64_t)cus * per_cu, std::max<int64_t>(ns, 1));
    TMCS_LAUNCH("k_bp", k_bp, dim3(bp_grid), dim3(bp_threads), bp_lds, stream, a);
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

void decode_release(Dem& D) {
  DecodeDevice* d = (DecodeDevice*)D.device;
  if (!d) return;
  free_device(d);
  delete d;
  D.device = nullptr;
}

}  // namespace tmcs
