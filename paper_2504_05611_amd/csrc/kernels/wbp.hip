// Weighted (neural) min-sum BP for training per-edge, per-iteration weights.
//
// Forward (T flooding iterations, no early stop):
//   m_t(c,v) = w_t(c,v) * sigma_t(c,v) * mu_t(c,v),  sigma = (-1)^{s_c} prod_{v'!=v} sgn q_{t-1},
//   mu = min_{v'!=v} |q_{t-1}| (1e30 if empty);  L_t = lambda + sum_c m_t;  q_t = L_t - m_t.
// It writes L_t for every t and, per iteration, the compressed check state
// (min1, min2, argmin edge, second argmin edge, sign parity, syndrome bit, one
// sign bit of q_{t-1} per edge).  The per-edge messages are not stored: the
// backward pass rebuilds them from that state.
//
// Backward, given G_t = dLoss/dL_t (reverse mode through the unrolled forward;
// the gradient of a min goes to the lowest-index edge attaining it, signs and
// the 1e30 of an empty minimum carry none):
//   gL_t(v) = G_t(v) + sum_c gq_t(v->c);  gm_t = gL_t(v) - gq_t(v->c);
//   dLoss/dw_t(c,v) = gm_t sigma_t mu_t;
//   gq_{t-1} at the argmin edge of each message += gm_t w_t sigma_t sgn(q_{t-1}).
// gq_t is nonzero only on each check's argmin and second-argmin edge, so it is
// carried as two numbers per check.
//
// A shot's working state lives in LDS, or (GS, when it exceeds the 160 KB of a
// compute unit, as for the surface-code CNOT at d >= 15) in a slab of device
// memory per workgroup with the same layout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../host/device.h"
#include "../host/timing.h"

namespace tmcs {

namespace {

constexpr float WBP_BIG = 1e30f;
constexpr int WBP_THREADS = 256;

struct WbpDevice {
  int device = -1;
  int32_t *row_ptr = nullptr, *col_idx = nullptr, *col_ptr = nullptr, *csc_row = nullptr, *csc_edge = nullptr;
  float* lam = nullptr;
  uint64_t* synd = nullptr;
  size_t cap_synd = 0;
  unsigned char* gstate = nullptr;   // GS: [grid][slab] per-workgroup state
  size_t cap_gstate = 0;
};

bool g_force_gs = false;             // keep the state in device memory even when it fits in LDS

// Per-iteration record in the workspace.
struct Layout {
  int64_t state;    // bytes of [m] float4-like {n1, n2, nag, a2}
  int64_t flags;    // bytes of [m] u8 (bit0 sign parity, bit1 syndrome), padded to 4
  int64_t signs;    // bytes of [nwords] u32
  int64_t iter;     // bytes per iteration
  int64_t shot;     // bytes per shot (T iterations)
};

Layout layout(const Dem& d, int T) {
  Layout L;
  const int64_t nwords = (d.edges + 31) / 32;
  L.state = (int64_t)d.rows * 16;
  L.flags = ((int64_t)d.rows + 3) / 4 * 4;
  L.signs = nwords * 4;
  L.iter = L.state + L.flags + L.signs;
  L.shot = L.iter * T;
  return L;
}

struct WbpArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* col_ptr;
  const int32_t* csc_row;
  const int32_t* csc_edge;
  const float* lam;
  const uint64_t* synd;      // [n_shots][mw]
  int32_t mw;
  int32_t m, n, T;
  int64_t E;
  int64_t nshots;
  const float* w;            // [T][E]
  float* llr;                // [T][n_shots][n]  (forward output)
  const float* gllr;         // [T][n_shots][n]  (backward input)
  float* gw;                 // [T][E]           (backward output, accumulated)
  unsigned char* ws;         // workspace
  Layout lay;
  unsigned char* gstate;     // GS: per-workgroup slabs
  int64_t slab;              // GS: bytes per slab
};

// 32-bit load from L2 (GS: the sign words are updated with atomics)
__device__ __forceinline__ uint32_t ld_sign(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool GS>
__global__ void __launch_bounds__(WBP_THREADS) k_wbp_forward(WbpArgs a) {
  extern __shared__ __align__(8) unsigned char sm[];
  unsigned char* base = GS ? a.gstate + (int64_t)blockIdx.x * a.slab : sm;
  const int tid = threadIdx.x;
  const int m = a.m, n = a.n;
  const int64_t nwords = (a.E + 31) / 32;
  auto sbit = [&](const uint32_t* es, int64_t e) -> int {
    return (int)(((GS ? ld_sign(&es[e >> 5]) : es[e >> 5]) >> (e & 31)) & 1u);
  };
  float* Lf = (float*)base;                              // [n]
  float* n1s = Lf + n;                                   // [m]
  float* n2s = n1s + m;                                  // [m]
  int32_t* ags = (int32_t*)(n2s + m);                    // [m]
  uint32_t* es = (uint32_t*)(ags + m);                   // [nwords]
  uint8_t* cf = (uint8_t*)(es + nwords);                 // [m]
  for (int64_t shot = blockIdx.x; shot < a.nshots; shot += gridDim.x) {
    const uint64_t* sy = a.synd + shot * a.mw;
    for (int c = tid; c < m; c += WBP_THREADS) {
      cf[c] = (uint8_t)(((sy[c >> 6] >> (c & 63)) & 1ull) << 1);
      n1s[c] = 0.0f;
      n2s[c] = 0.0f;
      ags[c] = -1;
    }
    for (int v = tid; v < n; v += WBP_THREADS) Lf[v] = a.lam[v];
    for (int64_t i = tid; i < nwords; i += WBP_THREADS) es[i] = 0u;
    __syncthreads();
    for (int t = 1; t <= a.T; ++t) {
      unsigned char* rec = a.ws + shot * a.lay.shot + (int64_t)(t - 1) * a.lay.iter;
      float* st = (float*)rec;
      uint8_t* fl_out = rec + a.lay.state;
      uint32_t* sg_out = (uint32_t*)(rec + a.lay.state + a.lay.flags);
      // check pass: q_{t-1} = L_{t-1} - m_{t-1}; new (min1, min2, argmin, 2nd argmin, parity)
      for (int c = tid; c < m; c += WBP_THREADS) {
        const int32_t r0 = a.row_ptr[c], r1 = a.row_ptr[c + 1];
        const float m1 = n1s[c], m2 = n2s[c];
        const int32_t ag = ags[c];
        const uint8_t fl = cf[c];
        const int sc = (fl >> 1) & 1, sp = fl & 1;
        float n1 = WBP_BIG, n2 = WBP_BIG;
        int32_t nag = -1, a2 = -1;
        int npar = 0;
        for (int32_t e = r0; e < r1; ++e) {
          const float Lv = Lf[a.col_idx[e]];
          const int se = sbit(es, e);
          const float wold = (t == 1) ? 1.0f : a.w[(int64_t)(t - 2) * a.E + e];
          const float mag = __fmul_rn(wold, e == ag ? m2 : m1);
          const float mo = (sc ^ sp ^ se) ? -mag : mag;
          const float q = __fsub_rn(Lv, mo);
          const float aq = fabsf(q);
          const int ng = q < 0.0f ? 1 : 0;
          if (aq < n1) { n2 = n1; a2 = nag; n1 = aq; nag = e; }
          else if (aq < n2) { n2 = aq; a2 = e; }
          npar ^= ng;
          if (ng != se) atomicXor(&es[e >> 5], 1u << (e & 31));
        }
        n1s[c] = n1;
        n2s[c] = n2;
        ags[c] = nag;
        cf[c] = (uint8_t)((sc << 1) | npar);
        st[4 * c + 0] = n1;
        st[4 * c + 1] = n2;
        ((int32_t*)st)[4 * c + 2] = nag;
        ((int32_t*)st)[4 * c + 3] = a2;
        fl_out[c] = (uint8_t)((sc << 1) | npar);
      }
      __syncthreads();
      for (int64_t i = tid; i < nwords; i += WBP_THREADS) sg_out[i] = GS ? ld_sign(&es[i]) : es[i];
      // variable pass: L_t = lambda + sum_c m_t (checks ascending)
      float* Lout = a.llr + ((int64_t)(t - 1) * a.nshots + shot) * n;
      for (int v = tid; v < n; v += WBP_THREADS) {
        float acc = a.lam[v];
        for (int32_t k = a.col_ptr[v]; k < a.col_ptr[v + 1]; ++k) {
          const int32_t c = a.csc_row[k], e = a.csc_edge[k];
          const uint8_t fl = cf[c];
          const int se = sbit(es, e);
          const float mag = __fmul_rn(a.w[(int64_t)(t - 1) * a.E + e], e == ags[c] ? n2s[c] : n1s[c]);
          const int neg = ((fl >> 1) ^ fl ^ se) & 1;
          acc = __fadd_rn(acc, neg ? -mag : mag);
        }
        Lf[v] = acc;
        Lout[v] = acc;
      }
      __syncthreads();
    }
  }
}

template <bool GS>
__global__ void __launch_bounds__(WBP_THREADS) k_wbp_backward(WbpArgs a) {
  extern __shared__ __align__(8) unsigned char sm[];
  unsigned char* base = GS ? a.gstate + (int64_t)blockIdx.x * a.slab : sm;
  const int tid = threadIdx.x;
  const int m = a.m, n = a.n;
  float* gL = (float*)base;                              // [n]
  float* g1n = gL + n;                                   // [m] gradient routed to argmin (next iteration)
  float* g2n = g1n + m;                                  // [m] ... to the second argmin
  int32_t* agn = (int32_t*)(g2n + m);                    // [m] argmin edges of the next iteration
  int32_t* a2n = agn + m;                                // [m]
  float* g1c = (float*)(a2n + m);                        // [m] current
  float* g2c = g1c + m;
  int32_t* agc = (int32_t*)(g2c + m);
  int32_t* a2c = agc + m;
  for (int64_t shot = blockIdx.x; shot < a.nshots; shot += gridDim.x) {
    for (int c = tid; c < m; c += WBP_THREADS) {
      g1n[c] = 0.0f;
      g2n[c] = 0.0f;
      agn[c] = -2;
      a2n[c] = -2;
    }
    __syncthreads();
    for (int t = a.T; t >= 1; --t) {
      const unsigned char* rec = a.ws + shot * a.lay.shot + (int64_t)(t - 1) * a.lay.iter;
      const float* st = (const float*)rec;
      const uint8_t* fl_in = rec + a.lay.state;
      const uint32_t* sg = (const uint32_t*)(rec + a.lay.state + a.lay.flags);
      const float* G = a.gllr + ((int64_t)(t - 1) * a.nshots + shot) * n;
      // gL_t(v) = G_t(v) + sum_c gq_t(v->c), routed by the next iteration's argmins
      for (int v = tid; v < n; v += WBP_THREADS) {
        float acc = G[v];
        for (int32_t k = a.col_ptr[v]; k < a.col_ptr[v + 1]; ++k) {
          const int32_t c = a.csc_row[k], e = a.csc_edge[k];
          if (e == agn[c]) acc += g1n[c];
          else if (e == a2n[c]) acc += g2n[c];
        }
        gL[v] = acc;
      }
      __syncthreads();
      // per check: dLoss/dw_t and the gradient reaching q_{t-1}
      for (int c = tid; c < m; c += WBP_THREADS) {
        const int32_t r0 = a.row_ptr[c], r1 = a.row_ptr[c + 1];
        const float n1 = st[4 * c + 0], n2 = st[4 * c + 1];
        const int32_t nag = ((const int32_t*)st)[4 * c + 2], a2 = ((const int32_t*)st)[4 * c + 3];
        const uint8_t fl = fl_in[c];
        const int sc = (fl >> 1) & 1, sp = fl & 1;
        float acc1 = 0.0f, acc2 = 0.0f;
        for (int32_t e = r0; e < r1; ++e) {
          const int32_t v = a.col_idx[e];
          const float gq = (e == agn[c]) ? g1n[c] : ((e == a2n[c]) ? g2n[c] : 0.0f);
          const float gm = gL[v] - gq;
          const int se = (int)((sg[e >> 5] >> (e & 31)) & 1u);
          const float sigma = (sc ^ sp ^ se) ? -1.0f : 1.0f;
          const float mu = e == nag ? n2 : n1;
          if (!(mu < WBP_BIG * 0.5f)) continue;
          atomicAdd(&a.gw[(int64_t)(t - 1) * a.E + e], gm * sigma * mu);
          const float ce = gm * a.w[(int64_t)(t - 1) * a.E + e] * sigma;
          if (e == nag) acc2 += ce; else acc1 += ce;
        }
        float g1 = 0.0f, g2 = 0.0f;
        if (nag >= 0) g1 = ((sg[nag >> 5] >> (nag & 31)) & 1u) ? -acc1 : acc1;
        if (a2 >= 0) g2 = ((sg[a2 >> 5] >> (a2 & 31)) & 1u) ? -acc2 : acc2;
        g1c[c] = g1;
        g2c[c] = g2;
        agc[c] = nag;
        a2c[c] = a2;
      }
      __syncthreads();
      for (int c = tid; c < m; c += WBP_THREADS) {
        g1n[c] = g1c[c];
        g2n[c] = g2c[c];
        agn[c] = agc[c];
        a2n[c] = a2c[c];
      }
      __syncthreads();
    }
  }
}

__global__ void k_wbp_transpose(const uint64_t* __restrict__ det, int32_t m, int64_t stride, int64_t nshots,
                                int32_t mw, uint64_t* __restrict__ synd) {
  __shared__ uint64_t tile[64];
  const int lane = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int rt = blockIdx.y;
  const int row = rt * 64 + lane;
  tile[lane] = row < m ? det[(int64_t)row * stride + w] : 0ull;
  __syncthreads();
  uint64_t out = 0ull;
  for (int i = 0; i < 64; ++i) out |= ((tile[i] >> lane) & 1ull) << i;
  const int64_t s = w * 64 + lane;
  if (s < nshots) synd[s * mw + rt] = out;
}

template <typename T>
tmcs_status upload(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
  if (hipMalloc((void**)dst, bytes) != hipSuccess) return fail(TMCS_ENOMEM, "hipMalloc failed (wbp)");
  if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(TMCS_EDEVICE, "hipMemcpy failed (wbp)");
  return TMCS_OK;
}

// The training kernels keep their own device copy of the graph (separate
// from the decoder's) in a static map keyed by the DEM handle.
struct Registry {
  std::vector<std::pair<const Dem*, WbpDevice*>> items;
};
Registry g_reg;

tmcs_status ensure(const Dem& D, WbpDevice** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TMCS_EDEVICE, "no HIP device");
  for (auto& it : g_reg.items)
    if (it.first == &D && it.second->device == dev) { *out = it.second; return TMCS_OK; }
  WbpDevice* d = new WbpDevice();
  d->device = dev;
  std::vector<float> lam(D.cols);
  for (int j = 0; j < D.cols; ++j) lam[j] = (float)std::log((1.0 - D.priors[j]) / D.priors[j]);
  std::vector<int32_t> csc_row(D.row_idx.begin(), D.row_idx.end());
  tmcs_status st;
  if ((st = upload(&d->row_ptr, D.row_ptr)) != TMCS_OK || (st = upload(&d->col_idx, D.col_idx)) != TMCS_OK ||
      (st = upload(&d->col_ptr, D.col_ptr)) != TMCS_OK || (st = upload(&d->csc_row, csc_row)) != TMCS_OK ||
      (st = upload(&d->csc_edge, D.csc_edge)) != TMCS_OK || (st = upload(&d->lam, lam)) != TMCS_OK)
    return st;
  g_reg.items.push_back({&D, d});
  *out = d;
  return TMCS_OK;
}

tmcs_status prepare(const Dem& D, int T, const uint64_t* det, uint64_t n_shots, WbpDevice** dd, WbpArgs* a,
                    hipStream_t stream) {
  WbpDevice* d = nullptr;
  tmcs_status st = ensure(D, &d);
  if (st != TMCS_OK) return st;
  const int mw = std::max((D.rows + 63) / 64, 1);
  const size_t need = (size_t)n_shots * mw;
  if (d->cap_synd < need) {
    hipFree(d->synd);
    d->synd = nullptr;
    d->cap_synd = 0;
    if (hipMalloc((void**)&d->synd, need * sizeof(uint64_t)) != hipSuccess) return fail(TMCS_ENOMEM, "hipMalloc (wbp syndromes)");
    d->cap_synd = need;
  }
  const int64_t stride = (int64_t)((n_shots + 63) / 64);
  TMCS_LAUNCH("k_wbp_transpose", k_wbp_transpose, dim3((unsigned)stride, (unsigned)mw), dim3(64), 0, stream, det,
              D.rows, stride, (int64_t)n_shots, mw, d->synd);
  WbpArgs& A = *a;
  A.row_ptr = d->row_ptr; A.col_idx = d->col_idx; A.col_ptr = d->col_ptr; A.csc_row = d->csc_row;
  A.csc_edge = d->csc_edge; A.lam = d->lam; A.synd = d->synd; A.mw = mw;
  A.m = D.rows; A.n = D.cols; A.T = T; A.E = D.edges; A.nshots = (int64_t)n_shots;
  A.lay = layout(D, T);
  *dd = d;
  return TMCS_OK;
}

// per-workgroup device-memory slabs of `bytes` each for the GS variants
tmcs_status slabs(WbpDevice* d, int grid, size_t bytes, WbpArgs* a) {
  const size_t slab = (bytes + 255) & ~(size_t)255;
  const size_t need = slab * (size_t)grid;
  if (d->cap_gstate < need) {
    hipFree(d->gstate);
    d->gstate = nullptr;
    d->cap_gstate = 0;
    if (hipMalloc((void**)&d->gstate, need) != hipSuccess) return fail(TMCS_ENOMEM, "hipMalloc (wbp state)");
    d->cap_gstate = need;
  }
  a->gstate = d->gstate;
  a->slab = (int64_t)slab;
  return TMCS_OK;
}

int grid_for(uint64_t n_shots) {
  int dev = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)n_shots, (int64_t)std::max(cus, 1) * 8));
}

}  // namespace

void wbp_set_global_state(bool on) { g_force_gs = on; }

size_t wbp_workspace_bytes(const Dem& d, int T, uint64_t n_shots) {
  return (size_t)layout(d, T).shot * (size_t)n_shots;
}

tmcs_status wbp_forward_run(const Dem& D, const float* w, int T, const uint64_t* det, uint64_t n_shots, float* llr,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
  if (n_shots == 0) return TMCS_OK;
  if (!det || !llr || !ws) return fail(TMCS_EINVAL, "null buffer");
  if (ws_bytes < wbp_workspace_bytes(D, T, n_shots)) return fail(TMCS_EINVAL, "workspace too small");
  WbpDevice* d = nullptr;
  WbpArgs a{};
  tmcs_status st = prepare(D, T, det, n_shots, &d, &a, stream);
  if (st != TMCS_OK) return st;
  a.w = w; a.llr = llr; a.ws = (unsigned char*)ws;
  const int64_t nwords = (D.edges + 31) / 32;
  const size_t lds = (size_t)D.cols * 4 + (size_t)D.rows * 13 + (size_t)nwords * 4 + 16;
  const int grid = grid_for(n_shots);
  if (g_force_gs || lds > 160 * 1024) {
    if ((st = slabs(d, grid, lds, &a)) != TMCS_OK) return st;
    TMCS_LAUNCH("k_wbp_forward", k_wbp_forward<true>, dim3(grid), dim3(WBP_THREADS), 0, stream, a);
    return hip_check(hipGetLastError(), "k_wbp_forward launch");
  }
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_wbp_forward<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return fail(TMCS_EUNSUPPORTED, "weighted BP state does not fit in LDS");
  TMCS_LAUNCH("k_wbp_forward", k_wbp_forward<false>, dim3(grid), dim3(WBP_THREADS), lds, stream, a);
  return hip_check(hipGetLastError(), "k_wbp_forward launch");
}

tmcs_status wbp_backward_run(const Dem& D, const float* w, int T, const uint64_t* det, uint64_t n_shots,
                             const float* gllr, float* gw, const void* ws, size_t ws_bytes, hipStream_t stream) {
  if (n_shots == 0) return TMCS_OK;
  if (!det || !ws) return fail(TMCS_EINVAL, "null buffer");
  if (ws_bytes < wbp_workspace_bytes(D, T, n_shots)) return fail(TMCS_EINVAL, "workspace too small");
  WbpDevice* d = nullptr;
  WbpArgs a{};
  tmcs_status st = prepare(D, T, det, n_shots, &d, &a, stream);
  if (st != TMCS_OK) return st;
  a.w = w; a.gllr = gllr; a.gw = gw; a.ws = (unsigned char*)ws;
  const size_t lds = (size_t)D.cols * 4 + (size_t)D.rows * 32 + 16;
  const int grid = grid_for(n_shots);
  if (g_force_gs || lds > 160 * 1024) {
    if ((st = slabs(d, grid, lds, &a)) != TMCS_OK) return st;
    TMCS_LAUNCH("k_wbp_backward", k_wbp_backward<true>, dim3(grid), dim3(WBP_THREADS), 0, stream, a);
    return hip_check(hipGetLastError(), "k_wbp_backward launch");
  }
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_wbp_backward<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return fail(TMCS_EUNSUPPORTED, "weighted BP state does not fit in LDS");
  TMCS_LAUNCH("k_wbp_backward", k_wbp_backward<false>, dim3(grid), dim3(WBP_THREADS), lds, stream, a);
  return hip_check(hipGetLastError(), "k_wbp_backward launch");
}

void wbp_release(const Dem& D) {
  for (size_t i = 0; i < g_reg.items.size(); ++i) {
    if (g_reg.items[i].first != &D) continue;
    WbpDevice* d = g_reg.items[i].second;
    hipFree(d->row_ptr); hipFree(d->col_idx); hipFree(d->col_ptr); hipFree(d->csc_row); hipFree(d->csc_edge);
    hipFree(d->lam); hipFree(d->synd);
    delete d;
    g_reg.items.erase(g_reg.items.begin() + i);
    --i;
  }
}

}  // namespace tmcs
