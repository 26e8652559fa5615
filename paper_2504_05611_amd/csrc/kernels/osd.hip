// OSD-0 (order-0 ordered-statistics decoding) and OSD-CS for the shots BP did
// not converge on: the elimination kernels and their launchers.  The decoder's
// BP side (decode.hip) hands over the FP32 posteriors of those shots through a
// device queue; see decode.hip for the whole pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "../host/device.h"
#include "../host/timing.h"
#include "decoder.h"

namespace tmcs {
namespace dec {



// Posteriors each thread has in flight in the selection passes: 8 in the
// windowed variant (hundreds of thousands of columns; 20-25 % faster there),
// 1 in the prefix variant (at most 16384 columns: the registers cost it a
// workgroup per SIMD, 50 % slower on BB [[144,12,12]] teleport).
template <bool WIN>
constexpr int sel_unroll() { return WIN ? 8 : 1; }

// Coherent (L2) 32-bit load: rowmap entries are updated with atomics and by
// other waves of the workgroup within one shot.
__device__ __forceinline__ int32_t ld_l2(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

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
// IDX32: store only the low 32 bits (the column index) of the sorted keys.
template <int KPT, bool IDX32 = false>
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
  for (int r = 0; r < KPT; ++r) {
    if (IDX32) ((uint32_t*)keys)[tid * KPT + r] = (uint32_t)x[r];
    else keys[tid * KPT + r] = x[r];
  }
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
// BL: the basis lives in LDS (after the sort keys) instead of HBM.
// NT: threads per workgroup (64: one wave decodes a shot on its own).
//
// WIN (DEMs beyond the dense limits): the scan that ends at the early stop only
// ever looks at a prefix of the sorted order, and those columns touch few rows.
// The shot therefore works on a window: the npad - 1 smallest keys at most
// (radix selection, then a sort), cut where the rows they touch would exceed
// win_rows, with those rows renumbered 0, 1, ... in order of first touch.  Kept
// columns are zero outside the window's rows, so independence tests, the early
// stop and the solution are exactly those of the full OSD-0 whenever s is
// spanned inside the window.  Otherwise (window too small) the shot keeps BP's
// hard decision and is flagged (flags bit 3, stats osd_incomplete).
//
// PFX (DEMs within the dense limits but wider than npad): the same selection
// gives the npad - 1 smallest keys, and the elimination runs on that prefix of
// the order with H's own rows.  If s is spanned there, the result is the full
// OSD-0's; otherwise the job goes to a retry list, which the full-sort variant
// then decodes, so every shot gets the exact OSD-0 correction.
//
// MULTI (windowed variant only): one launch serves the OSD queues of several
// decode items; job g of a counter shared by the launch belongs to item i with
// pref[i] <= g < pref[i + 1] (prefix sums of the items' queue lengths), and the
// workgroup switches to that item's arguments, basis and row table.  Every
// item's window has the same shape (npad = WIN_KEYS, 64 MW local rows), so the
// LDS layout does not change.
template <int MW, int RW, int KPT, bool BL, int NT, bool WIN = false, bool PFX = false, bool MULTI = false>
__global__ void __launch_bounds__(NT) k_osd(OSDArgs a, OSDMulti mu) {
  constexpr int W = MW + RW;
  static_assert(!(WIN && BL), "the window variant keeps its basis in HBM");
  static_assert(!(WIN && PFX), "one front end per variant");
  static_assert(!MULTI || WIN, "multi-item launches use the windowed variant");
  extern __shared__ __align__(8) unsigned char sm[];
  // local capacity: rank and rows of the problem the elimination sees
  const int cap_r = WIN ? 64 * MW : a.rank;
  const int cap_m = WIN ? 64 * MW : a.m;
  uint64_t* keys = (uint64_t*)sm;                                  // [npad] (BL, WIN: u32 column indices)
  uint64_t* lbasis = BL ? (uint64_t*)((uint32_t*)sm + a.npad) : keys + a.npad;   // BL: [rank][W]
  int32_t* pivot = (int32_t*)(BL ? lbasis + (size_t)a.rank * W : keys + a.npad);   // [rank] pivot row of basis i
  int32_t* kept = pivot + cap_r;                                   // [rank] column of basis i
  int32_t* prow = kept + cap_r;                                    // [m] basis index of a pivot row, or -1
  int32_t* srow = prow + cap_m;                                    // [m] rows with a syndrome bit
  // (an offset from sm, not an integer cast, so that the compiler keeps LDS addressing)
  const size_t acc_off = ((size_t)((unsigned char*)(srow + cap_m) - sm) + 7) & ~(size_t)7;
  uint64_t* acc = (uint64_t*)(sm + acc_off);                       // [W] solve accumulator
  uint32_t* tk = (uint32_t*)(acc + W);                             // OSD-CS: [npad / 32] kept sorted positions
  // WIN: after the sort, keys holds npad u32 column indices followed by npad
  // per-position counts (then exclusive offsets) of newly touched rows
  int32_t* pcnt = (int32_t*)keys + a.npad;
  __shared__ int s_job, s_r, s_ns, s_inc, s_inst;
  __shared__ int s_pref[MAX_MULTI_OSD + 1];
  __shared__ uint64_t s_red;
  __shared__ unsigned long long s_best;     // OSD-CS: (order key of the soft weight, candidate rank)
  __shared__ int s_tpos[64], s_nt, s_f1, s_f2;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  uint64_t* B = BL ? lbasis : a.basis + (int64_t)blockIdx.x * cap_r * W;
  int32_t* fpos = WIN ? a.rowmap + (int64_t)blockIdx.x * 2 * a.m : nullptr;   // [m] first window position
  int32_t* lmap = WIN ? fpos + a.m : nullptr;                                  // [m] local row index
  int cur = -1;                                                                // MULTI: current item
  if constexpr (MULTI) {
    if (tid == 0) {
      s_pref[0] = 0;
      for (int i = 0; i < mu.n; ++i) s_pref[i + 1] = s_pref[i] + mu.tab[i].counters[mu.tab[i].cnt_total];
    }
  }
  // acc = s + sum of the basis vectors pivoted on rows of s.  With a fully
  // reduced basis this is zero on every pivot row; its syndrome part is zero iff
  // s lies in the span of the kept columns, and its combination part then names
  // the kept columns whose sum is s.  Returns nonzero iff the syndrome part is.
  auto reduce_syndrome = [&]() {
    __syncthreads();
    if (tid < W) acc[tid] = 0ull;
    __syncthreads();
    for (int i = tid; i < s_ns; i += NT) {
      const int row = srow[i];
      atomicXor((unsigned long long*)&acc[row >> 6], (unsigned long long)(1ull << (row & 63)));
      const int pi = prow[row];
      if (pi >= 0) {
        const uint64_t* b = B + (int64_t)pi * W;
#pragma unroll
        for (int w = 0; w < W; ++w)
          if (b[w]) atomicXor((unsigned long long*)&acc[w], (unsigned long long)b[w]);
      }
    }
    __syncthreads();
    int nz = 0;
    for (int w = tid; w < MW; w += NT) nz |= acc[w] != 0ull;
    return __syncthreads_or(nz);
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
        s_job = atomicAdd(&a.counters[a.cnt_next], 1);
      }
    }
    __syncthreads();
    const int jn = s_job;
    if constexpr (MULTI) {
      const int inst = s_inst;
      __syncthreads();
      if (inst >= mu.n) break;
      if (inst != cur) {                     // uniform: the workgroup moves to the next item
        cur = inst;
        a = mu.tab[inst];
        B = a.basis + (int64_t)blockIdx.x * cap_r * W;
        fpos = a.rowmap + (int64_t)blockIdx.x * 2 * a.m;
        lmap = fpos + a.m;
      }
    } else {
      __syncthreads();
      if (jn >= a.counters[a.cnt_total]) break;
    }
    const int job = a.jobs ? a.jobs[jn] : jn;
    const int64_t ls = a.osd_queue[job];
    const int64_t shot = a.shot0 + ls;
    const float* L = a.osd_llr + (int64_t)job * a.n;
    int n_loc = a.n, rank_loc = a.rank, n0 = a.n;
    if (tid == 0) { s_r = 0; s_ns = 0; s_inc = 0; }
    __syncthreads();
    if constexpr (!WIN && !PFX) {
      // 1. sort columns by (L_v, v); list the syndrome's rows
      for (int r = tid; r < a.m; r += NT) prow[r] = -1;
      if (a.order > 0)
        for (int i = tid; i < (a.npad >> 5); i += NT) tk[i] = 0u;
      for (int wd = tid; wd < a.mw; wd += NT) {
        uint64_t x = a.synd[ls * a.mw + wd];
        if (x) {
          const int base = atomicAdd(&s_ns, __popcll(x));
          for (int k = 0; x; ++k, x &= x - 1) srow[base + k] = wd * 64 + (__ffsll((unsigned long long)x) - 1);
        }
      }
      uint64_t x[KPT];
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        const int i = tid * KPT + r;
        x[r] = i < a.n ? (((uint64_t)order_key(L[i]) << 32) | (uint32_t)i) : ~0ull;
      }
      bitonic_sort_regs<KPT, BL>(x, keys, a.npad);
    } else {
      __shared__ int s_hist[256];
      __shared__ int s_wsum[NT / 64];
      __shared__ int s_sel, s_want, s_cnt, s_cut, s_total;
      if (tid == 0) s_cnt = 0;
      __syncthreads();
      // 1a. the window: every key below the npad-th smallest 32-bit order key
      // (radix selection, 8 bits per pass), so at most npad - 1 columns, and all
      // of them when n < npad
      uint32_t kstar = 0xFFFFFFFFu;
      bool all = a.n < a.npad;
      if (!all) {
        uint32_t pre = 0u;
        int want = a.npad - 1;
        for (int pass = 0; pass < 4; ++pass) {
          const int sh = 24 - 8 * pass;
          const uint32_t hmask = pass == 0 ? 0u : (0xFFFFFFFFu << (sh + 8));
          for (int i = tid; i < 256; i += NT) s_hist[i] = 0;
          __syncthreads();
          // SEL_UNROLL posteriors per thread in flight (unconditional loads: the
          // last index is clamped and masked out afterwards)
          constexpr int SEL_UNROLL = sel_unroll<WIN>();
          for (int v0 = tid; v0 < a.n; v0 += NT * SEL_UNROLL) {
            uint32_t k[SEL_UNROLL];
#pragma unroll
            for (int i = 0; i < SEL_UNROLL; ++i) {
              const int v = v0 + i * NT;
              k[i] = order_key(L[v < a.n ? v : a.n - 1]);
            }
#pragma unroll
            for (int i = 0; i < SEL_UNROLL; ++i)
              if (v0 + i * NT < a.n && (k[i] & hmask) == (pre & hmask)) atomicAdd(&s_hist[(k[i] >> sh) & 255u], 1);
          }
          __syncthreads();
          if (wave == 0) {
            int c[4], t = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) { c[q] = s_hist[lane * 4 + q]; t += c[q]; }
            const int incl = wave_incl_scan(t);
            int e = incl - t;
            if (e <= want && want < incl) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                if (e <= want && want < e + c[q]) { s_sel = lane * 4 + q; s_want = want - e; }
                e += c[q];
              }
            }
          }
          __syncthreads();
          pre |= (uint32_t)s_sel << sh;
          want = s_want;
          __syncthreads();
        }
        kstar = pre;
      }
      // 1b. gather and sort the window's keys
      constexpr int SEL_UNROLL = sel_unroll<WIN>();
      for (int v0 = tid; v0 < a.n; v0 += NT * SEL_UNROLL) {
        uint32_t k[SEL_UNROLL];
#pragma unroll
        for (int i = 0; i < SEL_UNROLL; ++i) {
          const int v = v0 + i * NT;
          k[i] = order_key(L[v < a.n ? v : a.n - 1]);
        }
#pragma unroll
        for (int i = 0; i < SEL_UNROLL; ++i) {
          const int v = v0 + i * NT;
          if (v < a.n && (all || k[i] < kstar)) keys[atomicAdd(&s_cnt, 1)] = ((uint64_t)k[i] << 32) | (uint32_t)v;
        }
      }
      __syncthreads();
      n0 = s_cnt;
      uint64_t x[KPT];
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        const int i = tid * KPT + r;
        x[r] = i < n0 ? keys[i] : ~0ull;
      }
      bitonic_sort_regs<KPT, true>(x, keys, a.npad);
      const uint32_t* col32 = (const uint32_t*)keys;
      if constexpr (PFX) {
        // the prefix of the order, on H's rows
        n_loc = n0;
        for (int r = tid; r < a.m; r += NT) prow[r] = -1;
        for (int wd = tid; wd < a.mw; wd += NT) {
          uint64_t y = a.synd[ls * a.mw + wd];
          if (y) {
            const int base = atomicAdd(&s_ns, __popcll(y));
            for (int k = 0; y; ++k, y &= y - 1) srow[base + k] = wd * 64 + (__ffsll((unsigned long long)y) - 1);
          }
        }
        __syncthreads();
      } else {
      // 1c. first window position touching each row
      for (int j = tid; j < n0; j += NT) {
        const int col = (int)col32[j];
        for (int32_t k = a.col_ptr[col]; k < a.col_ptr[col + 1]; ++k) atomicMin(&fpos[a.csc_row[k]], j);
      }
      if (tid == 0) s_cut = n0;
      __syncthreads();
      // 1d. rows first touched at each position, exclusive offsets, and the cut:
      // the first position whose new rows would exceed win_rows
      int cnt[KPT], tsum = 0;
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        const int j = tid * KPT + r;
        cnt[r] = 0;
        if (j < n0) {
          const int col = (int)col32[j];
          for (int32_t k = a.col_ptr[col]; k < a.col_ptr[col + 1]; ++k) cnt[r] += ld_l2(&fpos[a.csc_row[k]]) == j;
        }
        tsum += cnt[r];
      }
      const int wincl = wave_incl_scan(tsum);
      if (lane == 63) s_wsum[wave] = wincl;
      __syncthreads();
      int off = wincl - tsum;
      for (int q = 0; q < wave; ++q) off += s_wsum[q];
      if (tid == NT - 1) s_total = off + tsum;
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        const int j = tid * KPT + r;
        if (j < n0) {
          pcnt[j] = off;
          if (off + cnt[r] > a.win_rows) atomicMin(&s_cut, j);
        }
        off += cnt[r];
      }
      __syncthreads();
      n_loc = s_cut;
      rank_loc = n_loc < n0 ? pcnt[n_loc] : s_total;      // rows of the window = bound on its rank
      // 1e. local row numbers, in order of first touch
      for (int j = tid; j < n_loc; j += NT) {
        const int col = (int)col32[j];
        int t = pcnt[j];
        for (int32_t k = a.col_ptr[col]; k < a.col_ptr[col + 1]; ++k) {
          const int r = a.csc_row[k];
          if (ld_l2(&fpos[r]) == j) __hip_atomic_store(&lmap[r], t++, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      for (int r = tid; r < rank_loc; r += NT) prow[r] = -1;
      __syncthreads();
      // 1f. the syndrome in local rows; a detection event outside the window
      // cannot be spanned by it
      for (int wd = tid; wd < a.mw; wd += NT) {
        uint64_t x = a.synd[ls * a.mw + wd];
        for (; x; x &= x - 1) {
          const int r = wd * 64 + (__ffsll((unsigned long long)x) - 1);
          if (ld_l2(&fpos[r]) >= n_loc) s_inc = 1;
          else srow[atomicAdd(&s_ns, 1)] = ld_l2(&lmap[r]);
        }
      }
      __syncthreads();
      }
    }
    // WIN, PFX: every column of H is in the window, so the result is the full OSD-0's
    const bool whole = !(WIN || PFX) || n_loc == a.n;
    const bool skip = WIN && !whole && s_inc;
    // rows of the elimination: H's, or the window's local numbers
    auto row_of = [&](int32_t k) -> int {
      const int r = a.csc_row[k];
      if constexpr (WIN) return ld_l2(&lmap[r]);
      else return r;
    };
    // 2. information set, 256 sorted candidates per pass (one per thread)
    for (int base = 0; base < (skip ? 0 : n_loc); base += NT) {
      const int r_start = s_r;
      __syncthreads();           // every wave has read s_r before wave 0 advances it
      if (r_start >= rank_loc) break;
      const int idx = base + tid;
      const int col = idx < n_loc ? ((BL || WIN || PFX) ? (int)((const uint32_t*)keys)[idx] : (int)(keys[idx] & 0xFFFFFFFFu)) : -1;
      uint64_t v[W];
#pragma unroll
      for (int w = 0; w < W; ++w) v[w] = 0ull;
      if (col >= 0) {
        const int32_t k0 = a.col_ptr[col], k1 = a.col_ptr[col + 1];
        for (int32_t k = k0; k < k1; ++k) {
          const int r = row_of(k);
#pragma unroll
          for (int w = 0; w < MW; ++w)
            if ((r >> 6) == w) v[w] ^= 1ull << (r & 63);
        }
        // phase 1: the basis vectors pivoted on rows of h
        for (int32_t k = k0; k < k1; ++k) {
          const int i = prow[row_of(k)];
          if (i >= 0) {
            const uint64_t* b = B + (int64_t)i * W;
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] ^= b[w];
          }
        }
      }
      __syncthreads();           // phase 1 everywhere before any wave publishes new pivots
      int r_done = r_start;
      for (int q = 0; q < NT / 64; ++q) {
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
          while (live && r < rank_loc) {
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
              if (!WIN && !PFX && a.order > 0) atomicOr(&tk[idx >> 5], 1u << (idx & 31));
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
          for (int i = tid; i < r_done; i += NT) {
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
      // Stop as soon as s lies in the span of the kept columns.  Columns of the
      // full information set are independent, so s has exactly one
      // representation over them; the one found here (zero on the columns not
      // yet kept) is it, and the rest of the scan could only add zeros.
      if ((WIN || PFX || a.order == 0) && !reduce_syndrome()) break;
    }
    // 3. solve: s reduced by the basis vectors pivoted on rows of s
    const int r = s_r;
    const int unspanned = skip ? 1 : reduce_syndrome();
    // WIN: a window that does not span s says nothing about H unless it is all of H
    const bool incomplete = unspanned && !whole;
    const int not_in_span = unspanned && whole;
    // the row table of a windowed shot is left all-sentinel for the next one
    auto reset_rows = [&]() {
      if constexpr (WIN) {
        const uint32_t* col32 = (const uint32_t*)keys;
        for (int j = tid; j < n0; j += NT) {
          const int col = (int)col32[j];
          for (int32_t k = a.col_ptr[col]; k < a.col_ptr[col + 1]; ++k)
            __hip_atomic_store(&fpos[a.csc_row[k]], WIN_NONE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    };
    if ((PFX || (WIN && a.retry)) && incomplete) {
      // PFX: the full sort decides this one; WIN with a retry list (the smaller
      // first window): the full window does
      if (tid == 0) a.retry[atomicAdd(&a.counters[4], 1)] = job;
      reset_rows();
      __syncthreads();
      continue;
    }
    if constexpr (!WIN && !PFX) {
      if (tid == 0) { s_f1 = -1; s_f2 = -1; }
      if (a.order > 0 && !not_in_span) {
        // OSD-CS: T = sorted positions not kept; candidates e_T of weight one over
        // T and of weight two over T's first `order` positions.  The soft weight of
        // a candidate sums L over e_S + rep(e_T) (kept columns in order of
        // selection) and then over e_T; the lightest wins, ties to the earlier.
        auto col_at = [&](int p) -> int {
          return BL ? (int)((const uint32_t*)keys)[p] : (int)(keys[p] & 0xFFFFFFFFu);
        };
        auto weight = [&](int c1, int c2) -> float {
          uint64_t x[RW];
#pragma unroll
          for (int w = 0; w < RW; ++w) x[w] = acc[MW + w];
          for (int q = 0; q < 2; ++q) {
            const int cc = q ? c2 : c1;
            if (cc < 0) continue;
            for (int32_t k = a.col_ptr[cc]; k < a.col_ptr[cc + 1]; ++k) {
              const int pi = prow[a.csc_row[k]];
              if (pi >= 0) {
                const uint64_t* bp = B + (int64_t)pi * W + MW;
#pragma unroll
                for (int w = 0; w < RW; ++w) x[w] ^= bp[w];
              }
            }
          }
          float c = 0.0f;
#pragma unroll
          for (int w = 0; w < RW; ++w)
            for (uint64_t y = x[w]; y; y &= y - 1) c = __fadd_rn(c, L[kept[w * 64 + (__ffsll((unsigned long long)y) - 1)]]);
          if (c1 >= 0) c = __fadd_rn(c, L[c1]);
          if (c2 >= 0) c = __fadd_rn(c, L[c2]);
          return c;
        };
        auto pair_of = [](int q, int nt, int* pa, int* pb) {
          int a0 = 0;
          while (q >= nt - 1 - a0) { q -= nt - 1 - a0; ++a0; }
          *pa = a0;
          *pb = a0 + 1 + q;
        };
        if (tid == 0) {
          int cnt = 0;
          for (int p = 0; p < n_loc && cnt < a.order; ++p)
            if (!((tk[p >> 5] >> (p & 31)) & 1u)) s_tpos[cnt++] = p;
          s_nt = cnt;
          s_best = ((unsigned long long)order_key(weight(-1, -1)) << 32);   // OSD-0 itself, rank 0
        }
        __syncthreads();
        unsigned long long best = ~0ull;
        for (int p = tid; p < n_loc; p += NT) {
          if ((tk[p >> 5] >> (p & 31)) & 1u) continue;
          const unsigned long long key = ((unsigned long long)order_key(weight(col_at(p), -1)) << 32) | (uint32_t)(1 + p);
          best = key < best ? key : best;
        }
        const int nt = s_nt, npairs = nt * (nt - 1) / 2;
        for (int q = tid; q < npairs; q += NT) {
          int ia, ib;
          pair_of(q, nt, &ia, &ib);
          const unsigned long long key = ((unsigned long long)order_key(weight(col_at(s_tpos[ia]), col_at(s_tpos[ib]))) << 32)
                                         | (uint32_t)(1 + a.npad + q);
          best = key < best ? key : best;
        }
        atomicMin(&s_best, best);
        __syncthreads();
        if (tid == 0) {
          const uint32_t rk = (uint32_t)(s_best & 0xFFFFFFFFu);
          int c1 = -1, c2 = -1;
          if (rk >= 1 && rk <= (uint32_t)a.npad) {
            c1 = col_at((int)rk - 1);
          } else if (rk > (uint32_t)a.npad) {
            int ia, ib;
            pair_of((int)rk - 1 - a.npad, nt, &ia, &ib);
            c1 = col_at(s_tpos[ia]);
            c2 = col_at(s_tpos[ib]);
          }
          for (int q = 0; q < 2; ++q) {
            const int cc = q ? c2 : c1;
            if (cc < 0) continue;
            for (int32_t k = a.col_ptr[cc]; k < a.col_ptr[cc + 1]; ++k) {
              const int pi = prow[a.csc_row[k]];
              if (pi >= 0)
                for (int w = 0; w < RW; ++w) acc[MW + w] ^= B[(int64_t)pi * W + MW + w];
            }
          }
          s_f1 = c1;
          s_f2 = c2;
        }
        __syncthreads();
      }
    }
    uint64_t pm[MAX_OW] = {0ull, 0ull, 0ull, 0ull};
    auto flip = [&](int col) {
      for (int w = 0; w < a.ow; ++w) pm[w] ^= a.obs_mask[(int64_t)w * a.n + col];
    };
    if (incomplete) {
      // BP's hard decision stands
      for (int v = tid; v < a.n; v += NT) {
        const bool e = L[v] < 0.0f;
        if (e) flip(v);
        if (a.ehat) a.ehat[shot * a.n + v] = e ? 1 : 0;
      }
    } else {
      if (a.ehat)
        for (int v = tid; v < a.n; v += NT) a.ehat[shot * a.n + v] = 0;
      __syncthreads();
      for (int i = tid; i < r; i += NT) {
        if ((acc[MW + (i >> 6)] >> (i & 63)) & 1ull) {
          const int col = kept[i];
          flip(col);
          if (a.ehat) a.ehat[shot * a.n + col] = 1;
        }
      }
      if constexpr (!WIN && !PFX) {
        // OSD-CS: the flipped columns outside the information set
        if (tid == 0)
          for (int q = 0; q < 2; ++q) {
            const int cc = q ? s_f2 : s_f1;
            if (cc < 0) continue;
            flip(cc);
            if (a.ehat) a.ehat[shot * a.n + cc] = 1;
          }
      }
    }
    for (int w = 0; w < a.ow; ++w) pm[w] = block_xor_u64(pm[w], &s_red);
    if (tid == 0) {
      for (int w = 0; w < a.ow; ++w) write_pred(a.pred, a.stride, a.nobs, shot, pm[w], w);
      if (a.flags) a.flags[shot] = (uint8_t)(2 | (not_in_span ? 4 : 0) | (incomplete ? 8 : 0));
      if (a.stats && not_in_span) atomicAdd((unsigned long long*)&a.stats->not_in_span, 1ull);
      if (a.stats && incomplete) atomicAdd((unsigned long long*)&a.stats->osd_incomplete, 1ull);
      if (a.stats && a.jobs) atomicAdd((unsigned long long*)&a.stats->osd_prefix_retry, 1ull);
    }
    reset_rows();
    __syncthreads();
  }
}

template <int MW, int RW, int KPT, bool BL, bool PFX = false>
tmcs_status launch_osd(const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  constexpr int NT = BL ? 64 : OSD_THREADS;
  auto k = k_osd<MW, RW, KPT, BL, NT, false, PFX>;
  if (lds > 64 * 1024 && hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return fail(TMCS_EUNSUPPORTED, "OSD workspace does not fit in LDS");
  // the full-sort pass over jobs a prefix left open is timed on its own
  TMCS_LAUNCH(a.jobs ? "k_osd_retry" : "k_osd", k, dim3(grid), dim3(NT), lds, s, a, OSDMulti{nullptr, 0, nullptr});
  return hip_check(hipGetLastError(), "k_osd launch");
}

// prefix pass: PFX_KEYS_WAVE (one wave) or PFX_KEYS_WG (256 threads) keys, 4 per thread
template <int MW>
tmcs_status launch_osd_pfx(bool bl, const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  // (one wave: at most PFX_KEYS_WAVE - 1 pivots, so PFX_KEYS_WAVE / 64 words of combination part)
  return bl ? launch_osd<MW, PFX_KEYS_WAVE / 64, PFX_KEYS_WAVE / 64, true, true>(a, grid, lds, s)
            : launch_osd<MW, MW, PFX_KEYS_WG / OSD_THREADS, false, true>(a, grid, lds, s);
}

tmcs_status dispatch_osd_pfx(int mw, bool bl, const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  if (bl) {
    if (mw <= 1) return launch_osd_pfx<1>(true, a, grid, lds, s);
    if (mw <= 2) return launch_osd_pfx<2>(true, a, grid, lds, s);
    if (mw <= 4) return launch_osd_pfx<4>(true, a, grid, lds, s);
    if (mw <= 5) return launch_osd_pfx<5>(true, a, grid, lds, s);
    if (mw <= 8) return launch_osd_pfx<8>(true, a, grid, lds, s);
    return fail(TMCS_EUNSUPPORTED, "OSD basis in LDS: too many detectors");
  }
  if (mw <= 1) return launch_osd_pfx<1>(false, a, grid, lds, s);
  if (mw <= 2) return launch_osd_pfx<2>(false, a, grid, lds, s);
  if (mw <= 4) return launch_osd_pfx<4>(false, a, grid, lds, s);
  if (mw <= 5) return launch_osd_pfx<5>(false, a, grid, lds, s);
  if (mw <= 8) return launch_osd_pfx<8>(false, a, grid, lds, s);
  if (mw <= 12) return launch_osd_pfx<12>(false, a, grid, lds, s);
  if (mw <= 15) return launch_osd_pfx<15>(false, a, grid, lds, s);
  if (mw <= 18) return launch_osd_pfx<18>(false, a, grid, lds, s);
  if (mw <= 24) return launch_osd_pfx<24>(false, a, grid, lds, s);
  if (mw <= 32) return launch_osd_pfx<32>(false, a, grid, lds, s);
  return fail(TMCS_EUNSUPPORTED, "OSD supports at most 2048 detectors in this build");
}

template <int MW>
tmcs_status dispatch_kpt(int kpt, const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (kpt) {
    case 1: return launch_osd<MW, MW, 1, false>(a, grid, lds, s);
    case 2: return launch_osd<MW, MW, 2, false>(a, grid, lds, s);
    case 4: return launch_osd<MW, MW, 4, false>(a, grid, lds, s);
    case 8: return launch_osd<MW, MW, 8, false>(a, grid, lds, s);
    case 16: return launch_osd<MW, MW, 16, false>(a, grid, lds, s);
    case 32: return launch_osd<MW, MW, 32, false>(a, grid, lds, s);
    case 64: return launch_osd<MW, MW, 64, false>(a, grid, lds, s);
    default: return fail(TMCS_EUNSUPPORTED, "OSD sort size");
  }
}

// basis in LDS, one wave per shot: small DEMs only (m <= 512, sort length <= 4096)
template <int MW>
tmcs_status dispatch_kpt_lds(int kpt, const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (kpt) {
    case 4: return launch_osd<MW, MW, 4, true>(a, grid, lds, s);
    case 8: return launch_osd<MW, MW, 8, true>(a, grid, lds, s);
    case 16: return launch_osd<MW, MW, 16, true>(a, grid, lds, s);
    case 32: return launch_osd<MW, MW, 32, true>(a, grid, lds, s);
    case 64: return launch_osd<MW, MW, 64, true>(a, grid, lds, s);
    default: return fail(TMCS_EUNSUPPORTED, "OSD sort size");
  }
}

bool osd_lds_basis_ok(int mw, int npad) { return mw <= 8 && npad <= 4096; }

// Windowed OSD-0 with 64 MW local rows.  A smaller window (WIN_SMALL_MW or
// WIN_MID_MW) runs first and hands the shots it cannot settle to a.retry; the full one
// (WIN_MW) decodes those (a.jobs = the retry list), timed as k_osd_retry.
template <int MW, bool MULTI>
tmcs_status launch_osd_win_t(const OSDArgs& a, const OSDMulti& mu, int grid, size_t lds, hipStream_t s) {
  auto k = k_osd<MW, MW, WIN_KEYS / OSD_THREADS, false, OSD_THREADS, true, false, MULTI>;
  if (lds > 64 * 1024 && hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return fail(TMCS_EUNSUPPORTED, "OSD workspace does not fit in LDS");
  TMCS_LAUNCH(a.jobs ? "k_osd_retry" : "k_osd", k, dim3(grid), dim3(OSD_THREADS), lds, s, a, mu);
  return hip_check(hipGetLastError(), "k_osd launch");
}

tmcs_status launch_osd_win(const OSDArgs& a, int grid, size_t lds, hipStream_t s, int mw) {
  const OSDMulti none{nullptr, 0, nullptr};
  if (mw == WIN_SMALL_MW) return launch_osd_win_t<WIN_SMALL_MW, false>(a, none, grid, lds, s);
  if (mw == WIN_MID_MW) return launch_osd_win_t<WIN_MID_MW, false>(a, none, grid, lds, s);
  if (mw == WIN_MW) return launch_osd_win_t<WIN_MW, false>(a, none, grid, lds, s);
  return fail(TMCS_EINVAL, "windowed OSD: unsupported window size");
}

tmcs_status launch_osd_win_multi(const OSDArgs& first, const OSDMulti& mu, int grid, size_t lds, hipStream_t s,
                                 int mw) {
  if (mu.n < 1 || mu.n > MAX_MULTI_OSD) return fail(TMCS_EINVAL, "multi-item OSD: 1..16 items");
  if (first.npad != WIN_KEYS) return fail(TMCS_EINVAL, "multi-item OSD: windowed items only");
  // the first item's arguments set the LDS layout, which every windowed item shares
  if (mw == WIN_SMALL_MW) return launch_osd_win_t<WIN_SMALL_MW, true>(first, mu, grid, lds, s);
  if (mw == WIN_MID_MW) return launch_osd_win_t<WIN_MID_MW, true>(first, mu, grid, lds, s);
  if (mw == WIN_MW) return launch_osd_win_t<WIN_MW, true>(first, mu, grid, lds, s);
  return fail(TMCS_EINVAL, "windowed OSD: unsupported window size");
}

tmcs_status dispatch_osd(int mw, int kpt, bool bl, const OSDArgs& a, int grid, size_t lds, hipStream_t s) {
  if (bl) {
    if (mw <= 1) return dispatch_kpt_lds<1>(kpt, a, grid, lds, s);
    if (mw <= 2) return dispatch_kpt_lds<2>(kpt, a, grid, lds, s);
    if (mw <= 4) return dispatch_kpt_lds<4>(kpt, a, grid, lds, s);
    if (mw <= 5) return dispatch_kpt_lds<5>(kpt, a, grid, lds, s);
    if (mw <= 8) return dispatch_kpt_lds<8>(kpt, a, grid, lds, s);
    return fail(TMCS_EUNSUPPORTED, "OSD basis in LDS: too many detectors");
  }
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

}  // namespace dec
}  // namespace tmcs
