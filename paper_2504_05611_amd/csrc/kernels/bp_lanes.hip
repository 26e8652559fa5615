// Min-sum BP for DEMs whose per-shot state does not fit in LDS: 64 shots per
// workgroup, one in each lane of every wave.
//
// The arithmetic is the one of the team kernel in decode.hip (same compressed
// state: L_v per column; min1, min2, argmin edge, sign parity and syndrome bit
// per check; one sign bit of q per edge), operation for operation, so both give
// bit-identical posteriors, iteration counts and decisions.  What differs is
// the layout of that state in device memory and who walks the Tanner graph:
//
//  - the state of the workgroup's 64 shots is interleaved by lane: check c's
//    record of lane j at [c][j] (16 B), L_v of lane j at [v][j] (4 B), and the
//    64 lanes' sign bits of edge e in one 64-bit word.  A wave touching check c
//    (or column v, or edge e) for its 64 shots reads or writes 1 KB (256 B, 8 B)
//    of consecutive bytes, so every access is a whole-line transfer;
//  - the waves split the checks (check pass) and the columns (variable pass)
//    between them: each wave walks its own record list, and all 64 lanes of a
//    wave run the same record, so records are wave-uniform (scalar registers)
//    and the lanes never diverge on the graph's irregular degrees;
//  - lanes keep their own iteration count: a lane whose shot converged (or ran
//    T iterations) takes the next shot of the queue at once, while the other
//    lanes go on.  A lane's first iteration reads the DEM's iteration-1 state
//    and its shot's syndrome bits directly instead of a copy of them;
//  - loads are issued LANES_UNROLL records at a time, so a wave keeps that many
//    independent line transfers in flight.
//
// The hard decision of every iteration folds the observable masks of the
// columns with L_v < 0 into a per-lane mask during the variable pass; a lane
// that converges therefore writes its prediction without another sweep.
// Shots handed to OSD copy their posteriors to the OSD staging rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "../host/device.h"
#include "../host/timing.h"
#include "decoder.h"

namespace tmcs {
namespace dec {

namespace {

constexpr int U = LANES_UNROLL;
constexpr int S = LANES_WAVES;

// A wave's record list is contiguous: lanes 0..4U-1 load the U records of a
// batch (one dword each) with one vector load, one batch ahead, and the batch's
// fields are then broadcast to scalar registers.
struct RecBatch {
  int v;                                   // this lane's dword of the batch
  __device__ __forceinline__ int4 rec(int u) const {
    return make_int4(__builtin_amdgcn_readlane(v, 4 * u), __builtin_amdgcn_readlane(v, 4 * u + 1),
                     __builtin_amdgcn_readlane(v, 4 * u + 2), __builtin_amdgcn_readlane(v, 4 * u + 3));
  }
};
__device__ __forceinline__ RecBatch rec_batch(const int* list, int k, int lane) {
  return RecBatch{list[(size_t)k * 4 + (lane & (4 * U - 1))]};   // (lanes past 4U repeat the batch)
}

template <bool WEIGHTED, bool MULTI>
__global__ void __launch_bounds__(64 * LANES_WAVES) k_bp_lanes(BPArgs a, BPMulti mu) {
  __shared__ int s_t[64];          // iteration the lane's shot is in (0: the lane has no shot)
  __shared__ int s_ls[64];         // the lane's shot (index into the chunk)
  __shared__ int s_f0[64];         // bit 0: s != 0; bit 1: a check without edges has s_c = 1
  __shared__ int s_pos[64], s_itr[64];
  __shared__ unsigned long long s_pm[64 * MAX_OW];
  __shared__ unsigned long long s_new, s_act, s_triv, s_unsat, s_fin, s_conv;
  __shared__ int s_exh;
  __shared__ unsigned long long s_cnt[4];   // nontrivial, converged, osd, iterations
  __shared__ unsigned long long s_hist[TMCS_BP_HIST_BINS];
  __shared__ unsigned long long s_pml[MAX_OW];   // the item's observables of the hard decision of lambda
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  int cur = 0;
  if constexpr (MULTI) a = mu.tab[0];
  float4* st4 = nullptr;
  float* Lb = nullptr;
  unsigned long long* sg = nullptr;
  int32_t total = 0;
  auto bind = [&]() {
    unsigned char* base = a.gstate + (size_t)blockIdx.x * a.team_bytes;
    st4 = (float4*)base;                                   // [m + 1][64] (row m: padding records)
    Lb = (float*)(st4 + (size_t)(a.m + 1) * 64);           // [n + 1][64] (row n: records that store no L)
    sg = (unsigned long long*)(Lb + (size_t)(a.n + 1) * 64);   // [E4 + 1] (word E4: padding records)
    total = a.queue ? a.counters[0] : (int32_t)a.nshots;
    if (tid == 0) {
#pragma unroll
      for (int w = 0; w < MAX_OW; ++w) s_pml[w] = a.pm_lam[w];
    }
  };
  bind();
  if (tid < 64) { s_t[tid] = 0; s_ls[tid] = 0; s_f0[tid] = 0; }
  if (tid < 4) s_cnt[tid] = 0ull;
  for (int i = tid; i < TMCS_BP_HIST_BINS; i += blockDim.x) s_hist[i] = 0ull;
  if (tid == 0) s_exh = 0;
  __syncthreads();
  // statistics of the current item to its stats block, then reset
  auto flush = [&]() {
    if (a.stats) {
      for (int i = tid; i < TMCS_BP_HIST_BINS; i += blockDim.x)
        if (s_hist[i]) atomicAdd((unsigned long long*)&a.stats->bp_iter_hist[i], s_hist[i]);
      if (tid == 0) {
        if (s_cnt[0]) atomicAdd((unsigned long long*)&a.stats->nontrivial, s_cnt[0]);
        if (s_cnt[1]) atomicAdd((unsigned long long*)&a.stats->converged, s_cnt[1]);
        if (s_cnt[2]) atomicAdd((unsigned long long*)&a.stats->osd, s_cnt[2]);
        if (s_cnt[3]) atomicAdd((unsigned long long*)&a.stats->bp_iters, s_cnt[3]);
      }
    }
    __syncthreads();
    for (int i = tid; i < TMCS_BP_HIST_BINS; i += blockDim.x) s_hist[i] = 0ull;
    if (tid < 4) s_cnt[tid] = 0ull;
    __syncthreads();
  };
  while (true) {
    // 1. lanes without a shot take the next ones of the queue
    if (wv == 0) {
      const bool idle = s_t[lane] == 0;
      const unsigned long long need = __ballot(idle);
      unsigned long long got = 0ull;
      if (need && !s_exh) {
        const int cnt = __popcll(need);
        int base = 0;
        if (lane == 0) base = atomicAdd(&a.counters[1], cnt);
        base = __shfl(base, 0, 64);
        const int idx = base + __popcll(need & ((1ull << lane) - 1ull));
        const bool take = idle && idx < total;
        if (take) {
          s_ls[lane] = a.queue ? a.queue[idx] : idx;
          s_t[lane] = 1;
          s_f0[lane] = (a.queue && !a.lone) ? 1 : 0;   // the compacted queue holds shots with s != 0 only
        }
        got = __ballot(take);
        if (lane == 0 && base + cnt >= total) s_exh = 1;
      }
      if (lane == 0) s_new = got;
    }
    __syncthreads();
    const unsigned long long nw = s_new;
    // 2. syndrome flags of the new shots, where the queue does not settle them
    if (nw && (!a.queue || a.lone)) {
      for (unsigned long long b = nw; b; b &= b - 1ull) {
        const int j = __ffsll((unsigned long long)b) - 1;
        const uint64_t* sy = a.synd + (int64_t)s_ls[j] * a.mw;
        int f = 0;
        for (int w = tid; w < a.mw; w += blockDim.x) {
          const uint64_t x = sy[w];
          f |= (x ? 1 : 0) | ((a.lone && (x & a.lone[w])) ? 2 : 0);
        }
        if (f) atomicOr(&s_f0[j], f);
      }
      __syncthreads();
    }
    // 3. the lanes that run an iteration now; a new shot with s = 0 ends at once (L = lambda)
    if (wv == 0) {
      const bool tv = ((nw >> lane) & 1ull) && !(s_f0[lane] & 1);
      const unsigned long long am = __ballot(s_t[lane] > 0 && !tv);
      const unsigned long long tm = __ballot(tv);
      if (lane == 0) { s_act = am; s_triv = tm; s_unsat = 0ull; }
      for (int w = 0; w < MAX_OW; ++w) s_pm[lane * MAX_OW + w] = 0ull;
    }
    __syncthreads();
    const unsigned long long act = s_act, trv = s_triv;
    if (!act && !trv) {
      // no lane holds a shot and the queue is empty
      if constexpr (MULTI) {
        flush();
        if (++cur >= mu.n) break;
        a = mu.tab[cur];
        bind();
        if (tid == 0) s_exh = 0;
        __syncthreads();
        continue;
      } else {
        break;
      }
    }
    if (act) {
      const bool on = (act >> lane) & 1ull;
      const int t = s_t[lane];
      const bool fresh = on && t == 1;
      const int f0 = s_f0[lane];
      const uint64_t* sy = a.synd + (int64_t)(fresh ? s_ls[lane] : 0) * a.mw;
      const bool use_w = WEIGHTED && a.w != nullptr;
      // weights of iteration t: the messages m^t of both passes
      const float* wt = use_w ? a.w + (int64_t)(t > 0 ? t - 1 : 0) * a.E : nullptr;
      // the item's fields the passes use, as locals
      const int m = a.m, n = a.n, E32 = a.E32, E4 = a.E4, ow = a.ow, Kv = a.Kv, Kc = a.Kc;
      const float alpha = a.alpha;
      const int4* init = a.init;
      const uint32_t* sign0w = a.sign0;                 // four sign bytes per word
      const uint64_t* obs_mask = a.obs_mask;
      // Loads of a batch are issued unconditionally (addresses chosen by selects),
      // so that no branch separates a load from its use and all of a batch's
      // loads are in flight together.  Lanes without a shot read their own slab
      // slots and discard the result.  A wave with a lane in its first iteration
      // runs the FRESH variant, which also reads the DEM's iteration-1 state.
      const bool wave_fresh = __ballot(fresh) != 0ull;
      const float* wsrc = use_w ? wt : a.lam;          // (unweighted: a valid address, value unused)
      // 4. variable pass: L^t from the state of iteration t, and the hard decision's observables
      auto vpass = [&](auto fresh_tag, auto owx_tag) {
        constexpr bool FRESH = decltype(fresh_tag)::value;
        constexpr bool OWX = decltype(owx_tag)::value;     // more than one observable word
        unsigned long long pm[MAX_OW] = {0ull, 0ull, 0ull, 0ull};
        float acc = 0.0f;
        const int* list = (const int*)(a.vsched + (size_t)wv * (Kv + U));
        RecBatch rb = rec_batch(list, 0, lane);
        for (int k = 0; k < Kv; k += U) {
          // the list holds U records of padding past its length, so the next batch is in bounds
          const RecBatch rbn = rec_batch(list, k + U, lane);
          int4 r[U];
#pragma unroll
          for (int u = 0; u < U; ++u) r[u] = rb.rec(u);
          // (a wave with a new shot takes the batch in halves: its loads need more registers)
          constexpr int UB = (FRESH || OWX) ? U / 2 : U;
          #pragma unroll
          for (int h = 0; h < U; h += UB) {
            float4 s[UB];
            unsigned long long g[UB], om[UB], omx[OWX ? UB : 1][MAX_OW - 1];
            float wv_[UB];
            int4 i0[UB];
            uint64_t sw[UB];
            uint32_t s0w[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
              const int v = r[h + u].x & R_IDX, e = r[h + u].y, c = r[h + u].z;
              s[u] = st4[(size_t)c * 64 + lane];
              g[u] = sg[e];
              om[u] = obs_mask[v];                      // observable word 0 (uniform address)
              if constexpr (OWX) {
                for (int w = 1; w < MAX_OW; ++w) omx[u][w - 1] = obs_mask[(size_t)(w < ow ? w : 0) * n + v];
              }
              if constexpr (WEIGHTED) wv_[u] = wsrc[use_w && e < E32 ? e : 0];
              if constexpr (FRESH) {
                const int cc = c < m ? c : m - 1;
                i0[u] = init[cc];
                sw[u] = sy[cc >> 6];
                s0w[u] = sign0w[(e < E4 ? e : E4 - 1) >> 2];
              }
            }
            int se[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
              se[u] = (int)((g[u] >> lane) & 1ull);
              if constexpr (FRESH) {
                const int c = r[h + u].z, e = r[h + u].y;
                const int cc = c < m ? c : m - 1;
                const int sb = (int)((sw[u] >> (cc & 63)) & 1ull);
                const float4 f = make_float4(__int_as_float(i0[u].x), __int_as_float(i0[u].y), __int_as_float(i0[u].z),
                                             __int_as_float(i0[u].w | (sb << 1)));
                const int ee = e < E4 ? e : E4 - 1;
                s[u] = fresh ? f : s[u];
                se[u] = fresh ? (int)((s0w[u] >> (8 * (ee & 3))) & 0xFFu) : se[u];
              }
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
              const int v = r[h + u].x & R_IDX, e = r[h + u].y;
              const float at = (WEIGHTED && use_w) ? wv_[u] : alpha;
              const float mag = __fmul_rn(at, e == __float_as_int(s[u].z) ? s[u].y : s[u].x);
              const int fl = __float_as_int(s[u].w);
              const float base = (r[h + u].x & R_FIRST) ? __int_as_float(r[h + u].w) : acc;   // lambda_v on a column's first edge
              acc = __fadd_rn(base, (((fl >> 1) ^ fl ^ se[u]) & 1) ? -mag : mag);
              // L_v on a column's last edge (other records write the spare row n),
              // and its observables into the hard decision's mask
              const bool last = (r[h + u].x & R_LAST) != 0;
              Lb[(size_t)(last ? v : n) * 64 + lane] = acc;
              const bool neg = last && acc < 0.0f;
              pm[0] ^= neg ? om[u] : 0ull;
              if constexpr (OWX) {
                for (int w = 1; w < MAX_OW; ++w) pm[w] ^= (neg && w < ow) ? omx[u][w - 1] : 0ull;
              }
            }
          }
          rb = rbn;
        }
        if (on) {
#pragma unroll
          for (int w = 0; w < MAX_OW; ++w)
            if (w < ow && pm[w]) atomicXor(&s_pm[lane * MAX_OW + w], pm[w]);
        }
      };
      if (ow > 1) {
        if (wave_fresh) vpass(std::true_type{}, std::true_type{});
        else vpass(std::false_type{}, std::true_type{});
      } else {
        if (wave_fresh) vpass(std::true_type{}, std::false_type{});
        else vpass(std::false_type{}, std::false_type{});
      }
      __syncthreads();
      // 5. check pass: H [L^t < 0] = s ?  and, if t < T, the state of iteration t + 1
      {
        const bool update = on && t < a.T;
        int unsat = (f0 >> 1) & 1;
        auto cpass = [&](auto fresh_tag) {
          constexpr bool FRESH = decltype(fresh_tag)::value;
          float n1o = 0.0f, n2o = 0.0f, n1 = BP_BIG, n2 = BP_BIG;
          int nago = -1, nag = -1, sc = 0, spo = 0, npar = 0, hard = 0;
          const int* list = (const int*)(a.csched + (size_t)wv * (Kc + U));
          RecBatch rb = rec_batch(list, 0, lane);
          for (int k = 0; k < Kc; k += U) {
            const RecBatch rbn = rec_batch(list, k + U, lane);
            int4 r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = rb.rec(u);
            constexpr int UB = FRESH ? U / 2 : U;
#pragma unroll
            for (int h = 0; h < U; h += UB) {
              float Lv[UB];
              unsigned long long g[UB];
              float4 s0[UB];
              float wv_[UB];
              int4 i0[UB];
              uint64_t sw[UB];
              uint32_t s0w[UB];
#pragma unroll
              for (int u = 0; u < UB; ++u) {
                const int v = r[h + u].x & R_IDX, e = r[h + u].y, c = r[h + u].z;
                const bool first = (r[h + u].x & R_FIRST) != 0;
                // a check's state is read on its first edge (records of one check are
                // consecutive, and every check's first record precedes its last); other
                // records read the padding row, which stays in cache
                s0[u] = st4[(size_t)(first ? c : m) * 64 + lane];
                Lv[u] = Lb[(size_t)v * 64 + lane];
                g[u] = sg[e];
                if constexpr (WEIGHTED) wv_[u] = wsrc[use_w && e < E32 ? e : 0];
                if constexpr (FRESH) {
                  const int cc = (first && c < m) ? c : 0;
                  i0[u] = init[cc];
                  sw[u] = sy[cc >> 6];
                  s0w[u] = sign0w[(e < E4 ? e : E4 - 1) >> 2];
                }
              }
#pragma unroll
              for (int u = 0; u < UB; ++u) {
                const int e = r[h + u].y, c = r[h + u].z;
                const bool first = (r[h + u].x & R_FIRST) != 0;
                int se = (int)((g[u] >> lane) & 1ull);
                if constexpr (FRESH) {
                  const int ee = e < E4 ? e : E4 - 1;
                  const int cc = (first && c < m) ? c : 0;
                  const int sb = (int)((sw[u] >> (cc & 63)) & 1ull);
                  const float4 f = make_float4(__int_as_float(i0[u].x), __int_as_float(i0[u].y), __int_as_float(i0[u].z),
                                               __int_as_float(i0[u].w | (sb << 1)));
                  se = fresh ? (int)((s0w[u] >> (8 * (ee & 3))) & 0xFFu) : se;
                  s0[u] = fresh ? f : s0[u];
                }
                {
                  const int fl = __float_as_int(s0[u].w);
                  n1o = first ? s0[u].x : n1o;
                  n2o = first ? s0[u].y : n2o;
                  nago = first ? __float_as_int(s0[u].z) : nago;
                  sc = first ? (fl >> 1) & 1 : sc;
                  spo = first ? fl & 1 : spo;
                }
                n1 = first ? BP_BIG : n1;
                n2 = first ? BP_BIG : n2;
                nag = first ? -1 : nag;
                npar = first ? 0 : npar;
                hard = (first ? 0 : hard) ^ (Lv[u] < 0.0f ? 1 : 0);
                // (lanes that do not update compute on whatever they read; nothing of theirs is stored)
                const float ao = (WEIGHTED && use_w) ? wv_[u] : alpha;
                const float mag = __fmul_rn(ao, e == nago ? n2o : n1o);
                const float q = __fsub_rn(Lv[u], (sc ^ spo ^ se) ? -mag : mag);   // q = L_v - m_old
                const float aq = fabsf(q);
                const int ng = q < 0.0f ? 1 : 0;
                const bool lt1 = aq < n1, lt2 = aq < n2;
                n2 = lt1 ? n1 : (lt2 ? aq : n2);
                n1 = lt1 ? aq : n1;
                nag = lt1 ? e : nag;
                npar ^= ng;
                // edge e's sign word: the bits of the lanes that update (the others'
                // bits are never read again: those lanes end their shot after this
                // pass); every lane stores the same word
                sg[e] = __ballot(update && ng != 0);
                // the check's new state on its last edge (other records, and lanes
                // that do not update, write the padding row m)
                const bool last = (r[h + u].x & R_LAST) != 0;
                unsat |= (last && on && hard != sc) ? 1 : 0;
                st4[(size_t)((last && update) ? c : m) * 64 + lane] =
                    make_float4(n1, n2, __int_as_float(nag), __int_as_float((sc << 1) | npar));
              }
            }
            rb = rbn;
          }
        };
        if (wave_fresh) cpass(std::true_type{});
        else cpass(std::false_type{});
        const unsigned long long ub = __ballot(on && unsat);
        if (lane == 0 && ub) atomicOr(&s_unsat, ub);
      }
      __syncthreads();
    }
    // 6. which lanes end their shot: converged, or T iterations without convergence
    if (wv == 0) {
      const int t = s_t[lane];
      const bool on = (act >> lane) & 1ull, tv = (trv >> lane) & 1ull;
      bool fin = tv, conv = tv;
      int itr = 0;
      if (on) {
        conv = !((s_unsat >> lane) & 1ull);
        fin = conv || t >= a.T;
        itr = conv ? t : a.T;
        if (!fin) s_t[lane] = t + 1;
      }
      const int pos = (fin && !conv && a.use_osd) ? atomicAdd(&a.counters[2], 1) : -1;
      s_pos[lane] = pos;
      s_itr[lane] = itr;
      const unsigned long long fm = __ballot(fin), cm = __ballot(fin && conv);
      if (lane == 0) { s_fin = fm; s_conv = cm; }
    }
    __syncthreads();
    // 7. ending lanes: posteriors to the OSD staging row (and per-shot outputs), predictions
    const unsigned long long fin = s_fin;
    if (fin) {
      const bool fl = (fin >> lane) & 1ull;
      const bool tv = (trv >> lane) & 1ull;
      const int pos = s_pos[lane];
      const int ls = s_ls[lane];
      const int64_t shot = a.shot0 + ls;
      const bool cp = fl && (pos >= 0 || a.llr != nullptr || a.ehat != nullptr);
      if (__ballot(cp)) {          // the same in every wave (it follows from shared values)
        constexpr int V = 8;
        for (int v0 = wv * V; v0 < a.n; v0 += S * V) {
          float Lv[V];
#pragma unroll
          for (int i = 0; i < V; ++i)
            Lv[i] = (cp && v0 + i < a.n) ? (tv ? a.lam[v0 + i] : Lb[(size_t)(v0 + i) * 64 + lane]) : 0.0f;
#pragma unroll
          for (int i = 0; i < V; ++i) {
            const int v = v0 + i;
            if (cp && v < a.n) {
              if (pos >= 0) a.osd_llr[(int64_t)pos * a.n + v] = Lv[i];
              if (a.llr) a.llr[shot * a.n + v] = Lv[i];
              if (a.ehat && pos < 0) a.ehat[shot * a.n + v] = Lv[i] < 0.0f ? 1 : 0;
            }
          }
        }
      }
      if (wv == 0 && fl) {
        const bool conv = (s_conv >> lane) & 1ull;
        const int itr = s_itr[lane];
        if (pos < 0) {
          for (int w = 0; w < a.ow; ++w)
            write_pred(a.pred, a.stride, a.nobs, shot, tv ? s_pml[w] : s_pm[lane * MAX_OW + w], w);
        } else {
          a.osd_queue[pos] = ls;
        }
        if (a.iters) a.iters[shot] = itr;
        if (a.flags) a.flags[shot] = (uint8_t)((conv ? 1 : 0) | (pos >= 0 ? 2 : 0));
        if (itr > 0 || !conv) atomicAdd(&s_cnt[0], 1ull);
        if (conv) atomicAdd(&s_cnt[1], 1ull);
        if (pos >= 0) atomicAdd(&s_cnt[2], 1ull);
        if (itr) atomicAdd(&s_cnt[3], (unsigned long long)itr);
        atomicAdd(&s_hist[itr < TMCS_BP_HIST_BINS - 1 ? itr : TMCS_BP_HIST_BINS - 1], 1ull);
        s_t[lane] = 0;
      }
    }
    __syncthreads();
  }
  if constexpr (!MULTI) flush();
}

}  // namespace

tmcs_status launch_bp_lanes(const BPArgs& a, const BPMulti& mu, bool weighted, int grid, hipStream_t s) {
  const dim3 g((unsigned)std::max(grid, 1)), b(64 * LANES_WAVES);
  if (mu.n > 0) {
    if (weighted) TMCS_LAUNCH("k_bp_lanes", (k_bp_lanes<true, true>), g, b, 0, s, a, mu);
    else TMCS_LAUNCH("k_bp_lanes", (k_bp_lanes<false, true>), g, b, 0, s, a, mu);
  } else {
    if (weighted) TMCS_LAUNCH("k_bp_lanes", (k_bp_lanes<true, false>), g, b, 0, s, a, mu);
    else TMCS_LAUNCH("k_bp_lanes", (k_bp_lanes<false, false>), g, b, 0, s, a, mu);
  }
  return hip_check(hipGetLastError(), "k_bp_lanes launch");
}

}  // namespace dec
}  // namespace tmcs
