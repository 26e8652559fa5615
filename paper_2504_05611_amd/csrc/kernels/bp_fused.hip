// Min-sum BP with one pass over the Tanner graph per iteration, for DEMs whose
// per-shot state lives in device memory.
//
// The flooding iteration t computes L^t_v = lambda_v + sum_c m^t(c->v) from the
// check state of iteration t, tests H [L^t < 0] = s, and builds the state of
// iteration t + 1 from q^{t+1}_{v->c} = L^t_v - m^t(c->v).  The team kernel in
// decode.hip does that in two passes (columns, then checks) with L^t stored in
// between.  Here a lane walks its checks only: for edge (c, v) it rebuilds
// L^t_v from the iteration-t states of v's checks, in the same order and with
// the same FP32 operations as the column pass (lambda_v first, then the
// messages of v's checks in ascending check order), so L^t, the decisions and
// the new state are bit-identical to the two-pass kernel's.  What it saves is
// the L array between the passes (a 4-byte write per column and a 4-byte read
// per edge), the second walk over the schedule and one workgroup barrier per
// iteration; what it pays is recomputing each message once more.
//
// The state of iteration t is read while that of t + 1 is written, so check
// records are double-buffered (iteration t reads buffer (t - 1) & 1), and each
// edge's sign byte holds sgn(q^t) in bit (t & 1) and receives sgn(q^{t+1}) in
// the other bit.  A sign byte is written only by the lane that owns its check;
// other lanes read the bit that write leaves unchanged.
//
// Schedule records, two int4 per edge, per-lane lists as in the check pass:
//   A = {v | R_FIRST | R_LAST (of the check), e, c, lambda_v bits}
//   B = {other check c' of v, its edge e', flags, 0} for a column of degree 2;
//       c' = -1: degree 1; c' = -2: degree >= 3, then y = first CSC index of v
//       and w = the degree.  flags bit 0: c' < c (c' first in the sum); bit 1:
//       c is v's first check (the edge that accounts for v's hard decision and
//       writes L_v when it is needed).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../host/device.h"
#include "../host/timing.h"
#include "decoder.h"

namespace tmcs {
namespace dec {

namespace {

// m^t(c -> v) for edge e of check c whose state is s, with sign bit se of q^t
__device__ __forceinline__ float message(float4 s, int e, int se, float at) {
  const float mag = __fmul_rn(at, e == __float_as_int(s.z) ? s.y : s.x);
  const int fl = __float_as_int(s.w);
  return (((fl >> 1) ^ fl ^ se) & 1) ? -mag : mag;
}

template <bool WEIGHTED, bool MULTI>
__global__ void __launch_bounds__(1024) k_bp_fused(BPArgs a, BPMulti mu) {
  __shared__ int s_job, s_flag, s_pos, s_inst;
  __shared__ int s_unsat;
  __shared__ int s_pref[MAX_MULTI + 1];
  __shared__ unsigned long long s_pm[MAX_OW];
  __shared__ unsigned long long s_hist[TMCS_BP_HIST_BINS];   // written by thread 0 only
  const int tid = threadIdx.x, P = blockDim.x;
  float4* st0 = nullptr;                                // [2][m + 1] check records (slot m: padding)
  float* L = nullptr;                                   // [n]
  uint8_t* sgn = nullptr;                               // [E4 + 4] (byte E4: padding records)
  auto bind = [&]() {
    unsigned char* base = a.gstate + (size_t)blockIdx.x * a.team_bytes;
    st0 = (float4*)base;
    L = (float*)(st0 + 2 * (size_t)(a.m + 1));
    sgn = (uint8_t*)(L + a.n);
  };
  int32_t total = 0;
  int cur = -1;
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
      s_unsat = 0;
    }
    __syncthreads();
    if constexpr (MULTI) {
      const int inst = s_inst;
      if (inst != cur) {                              // uniform: the team moves to the next item
        if (cur >= 0) flush();
        if (inst >= mu.n) break;
        cur = inst;
        a = mu.tab[inst];
        bind();
      }
    }
    const int job = s_job;
    if (!MULTI && job >= total) break;
    const bool use_w = WEIGHTED && (!MULTI || a.w != nullptr);
    const bool want_l = a.llr != nullptr || a.ehat != nullptr;   // L of every iteration (per-shot outputs)
    const int64_t ls = a.queue ? a.queue[job] : job;
    const int64_t shot = a.shot0 + ls;
    // state of iteration 1 (buffer 0), L = lambda, sgn(q^1) in bit 1 of each sign byte
    {
      const uint64_t* sy = a.synd + ls * a.mw;
      int fl = 0;
      for (int c = tid; c < a.m; c += P) {
        int4 s0 = a.init[c];
        const int sb = (int)((sy[c >> 6] >> (c & 63)) & 1ull);
        fl |= sb | ((s0.z < 0 && sb) ? 2 : 0);   // bit 1: a check without edges can never be satisfied
        s0.w |= sb << 1;
        st0[c] = make_float4(__int_as_float(s0.x), __int_as_float(s0.y), __int_as_float(s0.z), __int_as_float(s0.w));
      }
      for (int v = tid; v < a.n; v += P) L[v] = a.lam[v];
      // (sign bytes are 0 or 1: one shift moves every byte's bit 0 to bit 1)
      for (int i = tid; i < (a.E4 >> 2); i += P) ((uint32_t*)sgn)[i] = a.sign0[i] << 1;
      if (fl) atomicOr(&s_flag, fl);
    }
    __syncthreads();
    const int f0 = s_flag;
    int itr = 0;
    bool conv = true;
    if (f0 & 1) {
      conv = false;
      for (int t = 1;; ++t) {
        const float4* so = st0 + (size_t)((t - 1) & 1) * (a.m + 1);   // state of iteration t
        float4* sn = st0 + (size_t)(t & 1) * (a.m + 1);               // state of iteration t + 1
        const int ob = t & 1, nb = ob ^ 1;                             // sign bits of q^t and q^{t+1}
        const float* wt = use_w ? a.w + (int64_t)(t - 1) * a.E : nullptr;
        const bool update = t < a.T;
        const bool write_l = want_l || t == a.T;
        if (tid < MAX_OW) s_pm[tid] = 0ull;
        __syncthreads();
        int unsat = (f0 >> 1) & 1;
        uint64_t pm[MAX_OW] = {0ull, 0ull, 0ull, 0ull};
        float n1o = 0.0f, n2o = 0.0f, n1 = BP_BIG, n2 = BP_BIG;
        int nago = -1, nag = -1, sc = 0, spo = 0, npar = 0, hard = 0;
        auto step = [&](const int4 ra, const int4 rb) {
          const int v = ra.x & R_IDX, e = ra.y, c = ra.z;
          const bool first = (ra.x & R_FIRST) != 0;
          if (first) {
            const float4 s = so[c];
            const int fl = __float_as_int(s.w);
            n1o = s.x;
            n2o = s.y;
            nago = __float_as_int(s.z);
            sc = (fl >> 1) & 1;
            spo = fl & 1;
          }
          const int sbyte = sgn[e];
          const int se = (sbyte >> ob) & 1;
          const float at = use_w ? wt[e < a.E32 ? e : 0] : a.alpha;
          const float mag_own = __fmul_rn(at, e == nago ? n2o : n1o);
          const float m_own = ((sc ^ spo ^ se) & 1) ? -mag_own : mag_own;
          // L^t_v: lambda_v, then the messages of v's checks in ascending order
          const float lam = __int_as_float(ra.w);
          float Lv;
          if (rb.x >= 0) {
            const float4 s2 = so[rb.x];
            const int se2 = (sgn[rb.y] >> ob) & 1;
            const float at2 = use_w ? wt[rb.y < a.E32 ? rb.y : 0] : a.alpha;
            const float m2 = message(s2, rb.y, se2, at2);
            Lv = (rb.z & 1) ? __fadd_rn(__fadd_rn(lam, m2), m_own) : __fadd_rn(__fadd_rn(lam, m_own), m2);
          } else if (rb.x == -1) {
            Lv = __fadd_rn(lam, m_own);
          } else {
            Lv = lam;
            for (int j = rb.y; j < rb.y + rb.w; ++j) {
              const int c2 = a.csc_row[j], e2 = a.csc_edge[j];
              float m2;
              if (c2 == c) {
                m2 = m_own;
              } else {
                const float at2 = use_w ? wt[e2 < a.E32 ? e2 : 0] : a.alpha;
                m2 = message(so[c2], e2, (sgn[e2] >> ob) & 1, at2);
              }
              Lv = __fadd_rn(Lv, m2);
            }
          }
          n1 = first ? BP_BIG : n1;
          n2 = first ? BP_BIG : n2;
          nag = first ? -1 : nag;
          npar = first ? 0 : npar;
          hard = (first ? 0 : hard) ^ (Lv < 0.0f ? 1 : 0);
          if (rb.z & 2) {                               // v's first check: v's own bookkeeping
            if (Lv < 0.0f) {
#pragma unroll
              for (int w = 0; w < MAX_OW; ++w)
                if (w < a.ow) pm[w] ^= a.obs_mask[(int64_t)w * a.n + v];
            }
            if (write_l) L[v] = Lv;
          }
          if (update) {
            const float q = __fsub_rn(Lv, m_own);       // q^{t+1} = L^t_v - m^t(c->v)
            const float aq = fabsf(q);
            const int ng = q < 0.0f ? 1 : 0;
            const bool lt1 = aq < n1, lt2 = aq < n2;
            n2 = lt1 ? n1 : (lt2 ? aq : n2);
            n1 = lt1 ? aq : n1;
            nag = lt1 ? e : nag;
            npar ^= ng;
            sgn[e] = (uint8_t)((sbyte & (1 << ob)) | (ng << nb));
          }
          if (ra.x & R_LAST) {
            unsat |= hard != sc;
            if (update) sn[c] = make_float4(n1, n2, __int_as_float(nag), __int_as_float((sc << 1) | npar));
          }
        };
        // records are read two steps ahead; the schedule holds two rows of
        // padding past its (even) length, so every read is in bounds
        const int4* rp = a.fsched + 2 * (size_t)tid;
        const size_t stride = 2 * (size_t)P;
        int4 ra0 = rp[0], rb0 = rp[1], ra1 = rp[stride], rb1 = rp[stride + 1];
        for (int k = 0; k < a.Kf; k += 2) {
          step(ra0, rb0);
          ra0 = rp[(size_t)(k + 2) * stride];
          rb0 = rp[(size_t)(k + 2) * stride + 1];
          step(ra1, rb1);
          ra1 = rp[(size_t)(k + 3) * stride];
          rb1 = rp[(size_t)(k + 3) * stride + 1];
        }
        if (unsat) s_unsat = t;                           // benign race: every writer stores t
#pragma unroll
        for (int w = 0; w < MAX_OW; ++w)
          if (w < a.ow && pm[w]) atomicXor(&s_pm[w], (unsigned long long)pm[w]);
        __syncthreads();
        const bool still = s_unsat == t;
        if (!still) { itr = t; conv = true; break; }
        if (t >= a.T) { itr = a.T; break; }
      }
    }
    // finalize: prediction from the last hard decision, or hand the posteriors to OSD
    if (tid == 0) s_pos = (!conv && a.use_osd) ? atomicAdd(&a.counters[2], 1) : -1;
    __syncthreads();
    const int pos = s_pos;
    // (the pass accumulated the observables of its hard decision; a shot with
    // s = 0 ran no pass and its decision is lambda's)
    const bool from_pass = itr > 0;
    uint64_t pm[MAX_OW] = {0ull, 0ull, 0ull, 0ull};
    if (!from_pass || a.llr || a.ehat || pos >= 0)
      for (int v = tid; v < a.n; v += P) {
        const float Lv = L[v];
        if (!from_pass && pos < 0 && Lv < 0.0f) {
#pragma unroll
          for (int w = 0; w < MAX_OW; ++w)
            if (w < a.ow) pm[w] ^= a.obs_mask[(int64_t)w * a.n + v];
        }
        if (pos >= 0) a.osd_llr[(int64_t)pos * a.n + v] = Lv;
        if (a.llr) a.llr[shot * a.n + v] = Lv;
        if (a.ehat && pos < 0) a.ehat[shot * a.n + v] = Lv < 0.0f ? 1 : 0;
      }
    if (!from_pass) {
      if (tid < MAX_OW) s_pm[tid] = 0ull;
      __syncthreads();
#pragma unroll
      for (int w = 0; w < MAX_OW; ++w)
        if (w < a.ow && pm[w]) atomicXor(&s_pm[w], (unsigned long long)pm[w]);
    }
    __syncthreads();
    if (tid == 0) {
      if (pos < 0) {
        const uint64_t iso[MAX_OW] = {a.pm_iso[0], a.pm_iso[1], a.pm_iso[2], a.pm_iso[3]};
        for (int w = 0; w < a.ow; ++w) write_pred(a.pred, a.stride, a.nobs, shot, s_pm[w] ^ (from_pass ? iso[w] : 0ull), w);
      }
      else a.osd_queue[pos] = (int32_t)ls;
      if (a.iters) a.iters[shot] = itr;
      if (a.flags) a.flags[shot] = (uint8_t)((conv ? 1 : 0) | (pos >= 0 ? 2 : 0));
      c_nontriv += (itr > 0 || !conv) ? 1 : 0;
      c_conv += conv ? 1 : 0;
      c_osd += pos >= 0 ? 1 : 0;
      c_iters += (unsigned long long)itr;
      s_hist[itr < TMCS_BP_HIST_BINS - 1 ? itr : TMCS_BP_HIST_BINS - 1] += 1ull;
    }
    __syncthreads();
  }
  if constexpr (!MULTI) flush();
}

}  // namespace

tmcs_status launch_bp_fused(const BPArgs& a, const BPMulti& mu, bool weighted, int grid, int threads, hipStream_t s) {
  const dim3 g((unsigned)std::max(grid, 1)), b((unsigned)threads);
  if (mu.n > 0) {
    if (weighted) TMCS_LAUNCH("k_bp_dev", (k_bp_fused<true, true>), g, b, 0, s, a, mu);
    else TMCS_LAUNCH("k_bp_dev", (k_bp_fused<false, true>), g, b, 0, s, a, mu);
  } else {
    if (weighted) TMCS_LAUNCH("k_bp_dev", (k_bp_fused<true, false>), g, b, 0, s, a, mu);
    else TMCS_LAUNCH("k_bp_dev", (k_bp_fused<false, false>), g, b, 0, s, a, mu);
  }
  return hip_check(hipGetLastError(), "k_bp_fused launch");
}

}  // namespace dec
}  // namespace tmcs
