// Pauli-frame sampler for gfx950.
//
// Noise definition (the paper leaves the simulator's random bits open; this
// library fixes them so that every sampled bit is reproducible):
//   Philox4x32-10 (Salmon et al., SC'11) with key (seed lo, seed hi) and counter
//   (block b, site s, instance i, call j); the four words of call j are draws
//   4j..4j+3 of stream (b, s, i).  A block is 4096 consecutive shots.  With
//   T[k] = ceil((1-p)^k * 2^32) (FP64 product, k = 1..4096), a draw u gives the
//   number g = #{k : u < T[k]} of event-free shots before the next event; per
//   (b, s, i): pos = -1; repeat { pos += g(u) + 1; stop if pos >= 4096; event at
//   shot 4096 b + pos; for K-component channels draw v, component (v K) >> 32 }.
//   DEPOLARIZE1 component c is Pauli c+1 (X, Y, Z); DEPOLARIZE2 component c is
//   the pair (a, b) with c + 1 = 4a + b.
//
// Pipeline per chunk of blocks:
//   k_event_count  one thread per (block, site): length of its event stream
//   k_scan_*       exclusive prefix sum of the counts (block-major, site-minor)
//   k_event_write  one thread per (block, site): 64-bit events (position,
//                  component, channel kind, qubits)
//   k_frame        one workgroup per F consecutive 64-shot words of one block:
//                  X/Z frame words of every qubit live in LDS ([qubit][word],
//                  bit = shot), the layered program is executed with a barrier
//                  between layers, measurement records are XORed straight into
//                  detector/observable accumulator slots in LDS, and finished
//                  detectors are written to HBM as bit-packed words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <mutex>
#include <cmath>
#include <cstring>

#include "../host/device.h"
#include "../host/timing.h"
#include "../host/program.h"

namespace tmcs {

namespace {

constexpr int SB = 4096;          // shots per noise block
constexpr int WPB = SB / 64;      // 64-shot words per block
constexpr int FRAME_THREADS = 256;

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// g = #{k in 1..4096 : u < T[k]} with T non-increasing (tab[k-1] = T[k]).
// Since T[k] ~ (1-p)^k 2^32, g is close to log(u / 2^32) / log(1 - p); that
// value (inv = 1 / log(1 - p)) only picks where to start, and the table walk
// from there gives the exact count: T[g] > u >= T[g + 1].
__device__ __forceinline__ int geometric_gap(const uint64_t* __restrict__ tab, uint32_t u, double inv) {
  const uint64_t uu = u;
  if (inv == 0.0) return SB;                       // p = 0: T[k] = 2^32 > u for every k
  const double x = log(((double)u + 0.5) * (1.0 / 4294967296.0)) * inv;
  int k = x < 0.0 ? 0 : (x > (double)SB ? SB : (int)x);
  while (k < SB && __ldg(tab + k) > uu) ++k;
  while (k > 0 && __ldg(tab + k - 1) <= uu) --k;
  return k;
}

__device__ __forceinline__ int channel_k(uint8_t kind) {
  return kind == NK_DEP1 ? 3 : (kind == NK_DEP2 ? 15 : 1);
}

// Walk the event stream of (block, site); call emit(pos, comp) per event.
template <typename Emit>
__device__ __forceinline__ void event_stream(uint32_t k0, uint32_t k1, uint32_t block, uint32_t site,
                                             uint32_t inst, const uint64_t* __restrict__ tab, double inv, int K,
                                             Emit emit) {
  uint32_t w[4];
  uint32_t call = 0;
  int have = 0;
  int pos = -1;
  while (true) {
    if (have == 0) { philox4x32_10(block, site, inst, call++, k0, k1, w); have = 4; }
    const uint32_t u = w[4 - have--];
    pos += geometric_gap(tab, u, inv) + 1;
    if (pos >= SB) break;
    int comp = 0;
    if (K > 1) {
      if (have == 0) { philox4x32_10(block, site, inst, call++, k0, k1, w); have = 4; }
      const uint32_t v = w[4 - have--];
      comp = (int)(((uint64_t)v * (uint64_t)K) >> 32);
    }
    emit(pos, comp);
  }
}

__global__ void k_event_count(int64_t nsites, int64_t nblk, int64_t blk0, uint32_t k0, uint32_t k1,
                              uint32_t inst, const uint8_t* __restrict__ site_kind,
                              const uint16_t* __restrict__ site_tab, const uint64_t* __restrict__ tabs,
                              const double* __restrict__ tab_inv, uint32_t* __restrict__ counts,
                              const uint64_t* __restrict__ blk_off) {
  const int64_t n = nsites * nblk;
  if (blk_off) blk0 += (int64_t)*blk_off;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / nsites, s = i - b * nsites;
    const uint8_t kind = site_kind[s];
    uint32_t cnt = 0;
    const int ti = site_tab[s];
    event_stream(k0, k1, (uint32_t)(blk0 + b), (uint32_t)s, inst, tabs + (int64_t)ti * SB, tab_inv[ti],
                 channel_k(kind), [&](int, int) { ++cnt; });
    counts[i] = cnt;
  }
}

// Event word (64 bits): shot position in the block (12 bits), channel component
// (4), channel kind (2), first qubit (23) and second qubit + 1 (23; 0 = none).
__global__ void k_event_write(int64_t nsites, int64_t nblk, int64_t blk0, uint32_t k0, uint32_t k1,
                              uint32_t inst, const uint8_t* __restrict__ site_kind,
                              const uint16_t* __restrict__ site_tab, const uint64_t* __restrict__ tabs,
                              const double* __restrict__ tab_inv, const int2* __restrict__ site_q,
                              const uint32_t* __restrict__ offsets,
                              uint64_t* __restrict__ events, uint32_t capacity, uint32_t* __restrict__ overflow,
                              const uint64_t* __restrict__ blk_off) {
  const int64_t n = nsites * nblk;
  if (blk_off) blk0 += (int64_t)*blk_off;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / nsites, s = i - b * nsites;
    const uint8_t kind = site_kind[s];
    const int2 q = site_q[s];
    const uint64_t hi = ((uint64_t)kind << 16) | ((uint64_t)(uint32_t)q.x << 18) | ((uint64_t)(uint32_t)(q.y + 1) << 41);
    uint32_t o = offsets[i];
    const int ti = site_tab[s];
    event_stream(k0, k1, (uint32_t)(blk0 + b), (uint32_t)s, inst, tabs + (int64_t)ti * SB, tab_inv[ti],
                 channel_k(kind), [&](int pos, int comp) {
                   if (o < capacity) events[o] = hi | (uint64_t)(pos | (comp << 12));
                   else atomicOr(overflow, 1u);
                   ++o;
                 });
  }
}

// ---- exclusive scan of uint32 counts (3 kernels, 4096 items per workgroup)
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[SCAN_THREADS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t s = lane < SCAN_THREADS / 64 ? wsum[lane] : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < SCAN_THREADS / 64) wsum[lane] = s;
  }
  __syncthreads();
  const uint32_t base = wid ? wsum[wid - 1] : 0u;
  *total = wsum[SCAN_THREADS / 64 - 1];
  __syncthreads();
  return base + x - v;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_partials(const uint32_t* __restrict__ in, int64_t n,
                                                                uint32_t* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) s += base + k < n ? in[base + k] : 0u;
  uint32_t total;
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_top(uint32_t* __restrict__ partial, int64_t np) {
  uint32_t carry = 0;
  for (int64_t a = 0; a < np; a += SCAN_THREADS) {
    const int64_t i = a + threadIdx.x;
    const uint32_t v = i < np ? partial[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, &total);
    if (i < np) partial[i] = carry + ex;
    carry += total;
  }
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_final(const uint32_t* __restrict__ in, int64_t n,
                                                             const uint32_t* __restrict__ partial,
                                                             uint32_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) { v[k] = base + k < n ? in[base + k] : 0u; s += v[k]; }
  uint32_t total;
  uint32_t ex = block_exclusive_scan(s, &total) + partial[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k <= n) out[base + k] = ex;   // out has n + 1 entries
    ex += v[k];
  }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

struct FrameArgs {
  const int32_t* layers;     // [nlayers][3] kind, count, data offset (noise layers: noise ordinal)
  const int32_t* data;
  const int32_t* mslots;
  int32_t nlayers;
  int32_t Q;
  int32_t nslots;
  int32_t nsites;
  int32_t nnoise;            // noise layers
  const int32_t* noise_s0;   // [nnoise] first site of each noise layer (sites of a layer are consecutive)
  const int32_t* noise_cnt;  // [nnoise] sites in it
  const uint32_t* offsets;   // [chunk blocks * nsites + 1]
  const uint64_t* events;
  uint32_t capacity;
  int64_t blk0;              // first block of the chunk
  int64_t wg_word0;          // global word of workgroup 0's first word
  int64_t word_begin;        // global word of the call's first shot
  int64_t word_lo, word_hi;  // global words this launch covers [lo, hi)
  uint64_t shot_end;         // global shot end of the call
  uint64_t* det_out;
  uint64_t* obs_out;
  int64_t stride;            // words per output row
};

__device__ __forceinline__ int item_width(int32_t kind) {
  return (kind == L_RESET || kind == L_H || kind == L_CLEAR) ? 1 : (kind == L_CX || kind == L_EMIT) ? 2
         : kind == L_FEED ? 3 : 4;
}

// Operands of a thread's first PF items of one layer, loaded while the
// previous layer runs.
constexpr int PF = 4;
struct FramePrefetch {
  int32_t v[PF][4];          // gate layers: the item's integers
  uint64_t ev[PF];           // noise layers: event words
};

template <int F>
__device__ __forceinline__ void frame_prefetch(FramePrefetch& p, const FrameArgs& a, int L, const uint32_t* nl, int tid) {
  if (L >= a.nlayers) return;
  const int kind = a.layers[3 * L], cnt = a.layers[3 * L + 1], off = a.layers[3 * L + 2];
  if (kind == L_NOISE) {
    const uint32_t e0 = nl[2 * off], e1 = nl[2 * off + 1];
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const uint32_t e = e0 + tid + j * FRAME_THREADS;
      if (e < e1) p.ev[j] = a.events[e];
    }
    return;
  }
  const int w = item_width(kind);
  const int32_t* it = a.data + off;
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    const int g = (tid + j * FRAME_THREADS) / F;
    if (g < cnt) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (x < w) p.v[j][x] = it[w * g + x];
    }
  }
}

// One layer of the program on the F words of this workgroup.  Items of a layer
// touch distinct frame words (noise events of one site may share a word, hence
// the atomic XORs there; measurement records XOR into accumulator slots).
template <int F>
__device__ __forceinline__ void frame_layer(const FrameArgs& a, int L, const FramePrefetch& p, const uint32_t* nl,
                                            uint64_t* fx, uint64_t* fz, uint64_t* slot, int64_t gw0, int64_t blk,
                                            int wib0, int tid) {
  const int kind = a.layers[3 * L], cnt = a.layers[3 * L + 1], off = a.layers[3 * L + 2];
  if (kind == L_NOISE) {
    auto apply = [&](const uint64_t ev) {
      const int pos = (int)(ev & 4095u), comp = (int)((ev >> 12) & 15u), nk = (int)((ev >> 16) & 3u);
      const int q1 = (int)((ev >> 18) & 0x7FFFFFu), q2 = (int)((ev >> 41) & 0x7FFFFFu) - 1;
      const int f = (pos >> 6) - wib0;
      if (f < 0 || f >= F) return;
      const int64_t gw = gw0 + f;
      if (gw < a.word_lo || gw >= a.word_hi) return;
      if ((uint64_t)(blk * SB + pos) >= a.shot_end) return;
      const unsigned long long bit = 1ull << (pos & 63);
      int pa, pb = 0;
      if (nk == NK_XERR) pa = 1;
      else if (nk == NK_ZERR) pa = 3;
      else if (nk == NK_DEP1) pa = comp + 1;
      else { pa = (comp + 1) >> 2; pb = (comp + 1) & 3; }
      if (pa == 1 || pa == 2) atomicXor((unsigned long long*)&fx[q1 * F + f], bit);
      if (pa == 2 || pa == 3) atomicXor((unsigned long long*)&fz[q1 * F + f], bit);
      if (q2 >= 0) {
        if (pb == 1 || pb == 2) atomicXor((unsigned long long*)&fx[q2 * F + f], bit);
        if (pb == 2 || pb == 3) atomicXor((unsigned long long*)&fz[q2 * F + f], bit);
      }
    };
    const uint32_t e0 = nl[2 * off], e1 = nl[2 * off + 1];
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const uint32_t e = e0 + tid + j * FRAME_THREADS;
      if (e < e1) apply(p.ev[j]);
    }
    for (uint32_t e = e0 + tid + PF * FRAME_THREADS; e < e1; e += FRAME_THREADS) apply(a.events[e]);
    return;
  }
  const int w = item_width(kind);
  const int32_t* it = a.data + off;
  auto item = [&](const int g, const int f, const int32_t* v) {
    switch (kind) {
      case L_RESET:
        fx[v[0] * F + f] = 0ull;
        fz[v[0] * F + f] = 0ull;
        break;
      case L_H: {
        const uint64_t x = fx[v[0] * F + f];
        fx[v[0] * F + f] = fz[v[0] * F + f];
        fz[v[0] * F + f] = x;
        break;
      }
      case L_CX:
        fx[v[1] * F + f] ^= fx[v[0] * F + f];
        fz[v[0] * F + f] ^= fz[v[1] * F + f];
        break;
      case L_MEAS: {
        const uint64_t bit = v[1] ? fz[v[0] * F + f] : fx[v[0] * F + f];
        if (bit)
          for (int s2 = v[2]; s2 < v[3]; ++s2)
            atomicXor((unsigned long long*)&slot[a.mslots[s2] * F + f], (unsigned long long)bit);
        break;
      }
      case L_FEED: {
        const uint64_t x = slot[v[0] * F + f];
        if (v[2] == 1) fx[v[1] * F + f] ^= x;
        else fz[v[1] * F + f] ^= x;
        break;
      }
      case L_CLEAR:
        slot[v[0] * F + f] = 0ull;
        break;
      case L_EMIT: {
        const int64_t gw = gw0 + f;
        const uint64_t x = slot[v[0] * F + f];
        slot[v[0] * F + f] = 0ull;
        if (gw >= a.word_lo && gw < a.word_hi) {
          const int64_t col = gw - a.word_begin;
          if (v[1] >= 0) a.det_out[(int64_t)v[1] * a.stride + col] = x;
          else a.obs_out[(int64_t)(-v[1] - 1) * a.stride + col] = x;
        }
        break;
      }
      default:
        break;
    }
  };
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    const int i = tid + j * FRAME_THREADS;
    if (i < cnt * F) item(i / F, i % F, p.v[j]);
  }
  for (int i = tid + PF * FRAME_THREADS; i < cnt * F; i += FRAME_THREADS) {
    const int g = i / F;
    int32_t v[4] = {0, 0, 0, 0};
    for (int x = 0; x < w; ++x) v[x] = it[w * g + x];
    item(g, i % F, v);
  }
}

// One workgroup per F consecutive 64-shot words of one noise block.  The layer
// program runs with a barrier between layers; the next layer's operands are
// loaded into registers while the current one runs (two register sets that
// swap roles every layer).
template <int F>
__global__ void __launch_bounds__(FRAME_THREADS) k_frame(FrameArgs a) {
  extern __shared__ uint64_t smem[];
  uint64_t* fx = smem;
  uint64_t* fz = smem + (size_t)a.Q * F;
  uint64_t* slot = smem + (size_t)2 * a.Q * F;
  uint32_t* nl = (uint32_t*)(slot + (size_t)a.nslots * F);      // [nnoise][2] event range of each noise layer
  const int tid = threadIdx.x;
  const int64_t gw0 = a.wg_word0 + (int64_t)blockIdx.x * F;   // first global word of this WG
  const int64_t blk = gw0 / WPB;
  const int wib0 = (int)(gw0 - blk * WPB);                      // word-in-block of f = 0
  const int64_t ebase = (blk - a.blk0) * a.nsites;
  const int total = (2 * a.Q + a.nslots) * F;
  for (int i = tid; i < total; i += FRAME_THREADS) smem[i] = 0ull;
  for (int j = tid; j < a.nnoise; j += FRAME_THREADS) {
    const int s0 = a.noise_s0[j], c = a.noise_cnt[j];
    uint32_t e0 = a.offsets[ebase + s0], e1 = a.offsets[ebase + s0 + c];
    e0 = e0 < a.capacity ? e0 : a.capacity;
    e1 = e1 < a.capacity ? e1 : a.capacity;
    nl[2 * j] = e0;
    nl[2 * j + 1] = e1;
  }
  __syncthreads();
  FramePrefetch pa, pb;
  frame_prefetch<F>(pa, a, 0, nl, tid);
  for (int L = 0; L < a.nlayers; L += 2) {
    frame_prefetch<F>(pb, a, L + 1, nl, tid);
    frame_layer<F>(a, L, pa, nl, fx, fz, slot, gw0, blk, wib0, tid);
    __syncthreads();
    if (L + 1 >= a.nlayers) break;
    frame_prefetch<F>(pa, a, L + 2, nl, tid);
    frame_layer<F>(a, L + 1, pb, nl, fx, fz, slot, gw0, blk, wib0, tid);
    __syncthreads();
  }
}

struct SampleDevice {
  int device = -1;
  Program prog;
  int32_t* layers = nullptr;
  int32_t* data = nullptr;
  int32_t* mslots = nullptr;
  uint8_t* site_kind = nullptr;
  uint16_t* site_tab = nullptr;
  uint64_t* tabs = nullptr;
  double* tab_inv = nullptr;       // per table: 1 / log(1 - p) (search start only)
  int2* site_q = nullptr;          // per site: qubit(s) (second -1 for 1-qubit channels)
  int32_t* noise_s0 = nullptr;     // per noise layer: first site, number of sites
  int32_t* noise_cnt = nullptr;
  int32_t nnoise = 0;
  // scratch
  uint32_t* counts = nullptr;
  uint32_t* offsets = nullptr;
  uint32_t* partial = nullptr;
  uint64_t* events = nullptr;
  uint32_t* flag = nullptr;
  size_t cap_counts = 0, cap_offsets = 0, cap_partial = 0, cap_events = 0;
};

template <typename T>
tmcs_status upload(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
  if (hipMalloc((void**)dst, bytes) != hipSuccess) return fail(TMCS_ENOMEM, "hipMalloc failed (program)");
  if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(TMCS_EDEVICE, "hipMemcpy failed (program)");
  return TMCS_OK;
}

void free_device(SampleDevice* d) {
  hipFree(d->layers); hipFree(d->data); hipFree(d->mslots); hipFree(d->site_kind);
  hipFree(d->site_tab); hipFree(d->tabs); hipFree(d->counts); hipFree(d->offsets);
  hipFree(d->site_q); hipFree(d->noise_s0); hipFree(d->noise_cnt); hipFree(d->tab_inv);
  hipFree(d->partial); hipFree(d->events); hipFree(d->flag);
  *d = SampleDevice();
}

tmcs_status build_state(const Circuit& c, int dev, SampleDevice** out) {
  SampleDevice* d = new SampleDevice();
  d->device = dev;
  tmcs_status st = compile_program(c, &d->prog);
  if (st != TMCS_OK) { delete d; return st; }
  std::vector<uint64_t> tabs(d->prog.tab_p.size() * SB);
  std::vector<double> tab_inv(d->prog.tab_p.size());
  for (size_t i = 0; i < d->prog.tab_p.size(); ++i) {
    const double lq = std::log1p(-d->prog.tab_p[i]);
    tab_inv[i] = lq < 0.0 ? 1.0 / lq : 0.0;
    // T[k] = ceil(t_k 2^32), t_0 = 1, t_k = t_{k-1} (1 - p), FP64
    double t = 1.0;
    const double q = 1.0 - d->prog.tab_p[i];
    for (int k = 1; k <= SB; ++k) {
      t = t * q;
      tabs[i * SB + (k - 1)] = (uint64_t)std::ceil(t * 4294967296.0);
    }
  }
  // noise layers: their site ranges; the device copy of the layer table holds
  // the noise-layer ordinal in place of the data offset
  std::vector<int32_t> dlayers = d->prog.layers, ns0, ncnt;
  std::vector<int2> site_q(d->prog.site_kind.size(), make_int2(0, -1));
  for (int L = 0; L < d->prog.num_layers; ++L) {
    if (dlayers[3 * L] != L_NOISE) continue;
    const int cnt = dlayers[3 * L + 1], off = dlayers[3 * L + 2];
    const int32_t* it = d->prog.data.data() + off;
    for (int g = 0; g < cnt; ++g) {
      if (it[4 * g] != it[0] + g) { free_device(d); delete d; return fail(TMCS_EINVAL, "noise layer sites not consecutive"); }
      site_q[it[4 * g]] = make_int2(it[4 * g + 2], it[4 * g + 3]);
      if (it[4 * g + 2] >= (1 << 23) - 1 || it[4 * g + 3] >= (1 << 23) - 1) {
        free_device(d); delete d;
        return fail(TMCS_EUNSUPPORTED, "more than 2^23 - 1 qubits");
      }
    }
    dlayers[3 * L + 2] = (int32_t)ns0.size();
    ns0.push_back(it[0]);
    ncnt.push_back(cnt);
  }
  d->nnoise = (int32_t)ns0.size();
  if ((st = upload(&d->site_q, site_q)) != TMCS_OK || (st = upload(&d->noise_s0, ns0)) != TMCS_OK ||
      (st = upload(&d->noise_cnt, ncnt)) != TMCS_OK) {
    free_device(d);
    delete d;
    return st;
  }
  if ((st = upload(&d->layers, dlayers)) != TMCS_OK ||
      (st = upload(&d->data, d->prog.data)) != TMCS_OK ||
      (st = upload(&d->mslots, d->prog.mslots)) != TMCS_OK ||
      (st = upload(&d->site_kind, d->prog.site_kind)) != TMCS_OK ||
      (st = upload(&d->site_tab, d->prog.site_tab)) != TMCS_OK ||
      (st = upload(&d->tabs, tabs)) != TMCS_OK || (st = upload(&d->tab_inv, tab_inv)) != TMCS_OK) {
    free_device(d);
    delete d;
    return st;
  }
  if (hipMalloc((void**)&d->flag, sizeof(uint32_t)) != hipSuccess) {
    free_device(d);
    delete d;
    return fail(TMCS_ENOMEM, "hipMalloc failed (flag)");
  }
  *out = d;
  return TMCS_OK;
}

// The device state cached on the circuit handle (rebuilt when the device changes).
tmcs_status ensure_device(const Circuit& cc, SampleDevice** out) {
  Circuit& c = const_cast<Circuit&>(cc);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TMCS_EDEVICE, "no HIP device");
  SampleDevice* d = (SampleDevice*)c.device;
  if (d && d->device == dev) { *out = d; return TMCS_OK; }
  if (d) { free_device(d); delete d; c.device = nullptr; }
  tmcs_status st = build_state(c, dev, &d);
  if (st != TMCS_OK) return st;
  c.device = d;
  *out = d;
  return TMCS_OK;
}

template <typename T>
tmcs_status grow(T** p, size_t* cap, size_t need) {
  if (*cap >= need) return TMCS_OK;
  hipFree(*p);
  *p = nullptr;
  *cap = 0;
  const size_t n = need + need / 4 + 1024;
  if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) return fail(TMCS_ENOMEM, "hipMalloc failed (sampler scratch)");
  *cap = n;
  return TMCS_OK;
}

int frame_words_per_wg(const Program& P, int Q, int nnoise, size_t* lds_bytes) {
  const size_t per_word = (size_t)(2 * Q + P.nslots) * sizeof(uint64_t);
  const size_t fixed = (size_t)nnoise * 8;
  int F = 64;
  while (F > 1 && per_word * F + fixed > 64 * 1024) F >>= 1;
  *lds_bytes = per_word * F + fixed;
  return F;
}

template <int F>
tmcs_status launch_frame(const FrameArgs& a, int64_t nwg, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024) {
    if (hipFuncSetAttribute((const void*)k_frame<F>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return fail(TMCS_EUNSUPPORTED, "frame does not fit in LDS");
  }
  TMCS_LAUNCH("k_frame", k_frame<F>, dim3((unsigned)nwg), dim3(FRAME_THREADS), lds, s, a);
  return hip_check(hipGetLastError(), "k_frame launch");
}

// Scratch of the no-allocation sampler (tmcs_sample_noalloc): a file-scope
// device array, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel: it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[64] = {};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of event scratch for a chunk of nblk blocks: counts and offsets
// (n + 1 each), scan partials, and the event buffer (its capacity as below).
size_t chunk_scratch_bytes(int64_t nsites, int64_t nblk, double events_per_shot, size_t* cap_out) {
  const int64_t n = nblk * nsites;
  const double mean = events_per_shot * (double)(nblk * SB);
  const size_t cap = (size_t)(mean * 1.25 + 16.0 * std::sqrt(mean) + 65536.0);
  const int64_t ntiles = (n + 1 + SCAN_TILE - 1) / SCAN_TILE;
  if (cap_out) *cap_out = cap;
  return 2 * align256((size_t)(n + 1) * 4) + align256((size_t)(ntiles + 1) * 4) + align256(cap * 8);
}

}  // namespace

tmcs_status sample_run(const Circuit& c, uint64_t seed, uint32_t instance, uint64_t shot_begin,
                       uint64_t n_shots, uint64_t* det, uint64_t* obs, hipStream_t stream,
                       const uint64_t* blk_off, uint32_t* overflow_out, void* state,
                       unsigned char* fixed, size_t fixed_bytes) {
  if (shot_begin % 64) return fail(TMCS_EINVAL, "shot_begin must be a multiple of 64");
  if (n_shots == 0) return TMCS_OK;
  if ((c.num_dets && !det) || (c.num_obs && !obs)) return fail(TMCS_EINVAL, "null output buffer");
  if ((shot_begin + n_shots) / SB >= (1ull << 32)) return fail(TMCS_EINVAL, "shot index beyond 2^44");
  SampleDevice* d = (SampleDevice*)state;
  tmcs_status st = TMCS_OK;
  if (!d && (st = ensure_device(c, &d)) != TMCS_OK) return st;
  const Program& P = d->prog;
  const int64_t nsites = (int64_t)P.site_kind.size();
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  const uint64_t shot_end = shot_begin + n_shots;
  const int64_t stride = (int64_t)((n_shots + 63) / 64);
  const int64_t word_begin = (int64_t)(shot_begin / 64);
  size_t lds = 0;
  const int F = frame_words_per_wg(P, c.num_qubits, d->nnoise, &lds);
  if (lds > 160 * 1024) return fail(TMCS_EUNSUPPORTED, "circuit frame exceeds the 160 KB LDS of one workgroup");
  // the overflow flag: per call, or a caller-owned sticky flag (graph replays)
  uint32_t* flag = overflow_out ? overflow_out : d->flag;
  if (!overflow_out) TMCS_LAUNCH("k_zero_u32", k_zero_u32, dim3(1), dim3(64), 0, stream, flag, 1);
  // chunk of blocks: bound the per-(block, site) arrays to ~64M entries
  const int64_t blk_first = (int64_t)(shot_begin / SB);
  const int64_t blk_last = (int64_t)((shot_end - 1) / SB);
  int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(256, (64ll << 20) / std::max<int64_t>(nsites, 1)));
  if (fixed) {
    // the largest chunk whose scratch fits the caller-provided area
    if (chunk_scratch_bytes(nsites, 1, P.events_per_shot, nullptr) > fixed_bytes)
      return fail(TMCS_EUNSUPPORTED, "this circuit needs " +
                  std::to_string(chunk_scratch_bytes(nsites, 1, P.events_per_shot, nullptr)) +
                  " bytes of event scratch per 4096-shot block; the no-allocation scratch holds " +
                  std::to_string(fixed_bytes));
    while (chunk > 1 && chunk_scratch_bytes(nsites, chunk, P.events_per_shot, nullptr) > fixed_bytes)
      chunk = std::max<int64_t>(1, chunk / 2);
  }
  for (int64_t b0 = blk_first; b0 <= blk_last; b0 += chunk) {
    const int64_t b1 = std::min(blk_last + 1, b0 + chunk);
    const int64_t nblk = b1 - b0;
    const uint64_t s_lo = std::max<uint64_t>(shot_begin, (uint64_t)b0 * SB);
    const uint64_t s_hi = std::min<uint64_t>(shot_end, (uint64_t)b1 * SB);
    const int64_t n = nblk * nsites;
    const double mean = P.events_per_shot * (double)(nblk * SB);
    const size_t cap = (size_t)(mean * 1.25 + 16.0 * std::sqrt(mean) + 65536.0);
    if (cap >= 0xFFFFFFF0ull) return fail(TMCS_EUNSUPPORTED, "too many noise events per chunk");
    const int64_t ntiles = (n + 1 + SCAN_TILE - 1) / SCAN_TILE;
    uint32_t *counts, *offsets, *partial;
    uint64_t* events;
    size_t cap_events;
    if (fixed) {
      counts = (uint32_t*)fixed;
      offsets = (uint32_t*)(fixed + align256((size_t)(n + 1) * 4));
      partial = (uint32_t*)(fixed + 2 * align256((size_t)(n + 1) * 4));
      events = (uint64_t*)(fixed + 2 * align256((size_t)(n + 1) * 4) + align256((size_t)(ntiles + 1) * 4));
      cap_events = cap;
    } else {
      if ((st = grow(&d->counts, &d->cap_counts, (size_t)n + 1)) != TMCS_OK ||
          (st = grow(&d->offsets, &d->cap_offsets, (size_t)n + 1)) != TMCS_OK ||
          (st = grow(&d->partial, &d->cap_partial, (size_t)ntiles + 1)) != TMCS_OK ||
          (st = grow(&d->events, &d->cap_events, cap)) != TMCS_OK)
        return st;
      counts = d->counts; offsets = d->offsets; partial = d->partial; events = d->events;
      cap_events = d->cap_events;
    }
    if (nsites > 0) {
      const int thr = 256;
      const int64_t grid = std::min<int64_t>((n + thr - 1) / thr, 1 << 20);
      TMCS_LAUNCH("k_event_count", k_event_count, dim3((unsigned)grid), dim3(thr), 0, stream, nsites, nblk, b0, k0, k1,
                         instance, d->site_kind, d->site_tab, d->tabs, d->tab_inv, counts, blk_off);
      TMCS_LAUNCH("k_scan_partials", k_scan_partials, dim3((unsigned)ntiles), dim3(SCAN_THREADS), 0, stream, counts, n, partial);
      TMCS_LAUNCH("k_scan_top", k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, stream, partial, ntiles);
      TMCS_LAUNCH("k_scan_final", k_scan_final, dim3((unsigned)ntiles), dim3(SCAN_THREADS), 0, stream, counts, n, partial, offsets);
      TMCS_LAUNCH("k_event_write", k_event_write, dim3((unsigned)grid), dim3(thr), 0, stream, nsites, nblk, b0, k0, k1,
                         instance, d->site_kind, d->site_tab, d->tabs, d->tab_inv, d->site_q, offsets, events,
                         (uint32_t)cap_events, flag, blk_off);
      if ((st = hip_check(hipGetLastError(), "event kernels")) != TMCS_OK) return st;
    }
    FrameArgs a;
    a.layers = d->layers; a.data = d->data; a.mslots = d->mslots;
    a.nlayers = P.num_layers; a.Q = c.num_qubits; a.nslots = P.nslots; a.nsites = (int32_t)nsites;
    a.nnoise = d->nnoise; a.noise_s0 = d->noise_s0; a.noise_cnt = d->noise_cnt;
    a.offsets = offsets; a.events = events; a.capacity = (uint32_t)cap_events;
    a.blk0 = b0;
    a.word_lo = (int64_t)(s_lo / 64);
    a.word_hi = (int64_t)((s_hi + 63) / 64);
    a.wg_word0 = (a.word_lo / F) * F;
    a.word_begin = word_begin;
    a.shot_end = shot_end;
    a.det_out = det; a.obs_out = obs; a.stride = stride;
    const int64_t nwg = (a.word_hi - a.wg_word0 + F - 1) / F;
    switch (F) {
      case 64: st = launch_frame<64>(a, nwg, lds, stream); break;
      case 32: st = launch_frame<32>(a, nwg, lds, stream); break;
      case 16: st = launch_frame<16>(a, nwg, lds, stream); break;
      case 8: st = launch_frame<8>(a, nwg, lds, stream); break;
      case 4: st = launch_frame<4>(a, nwg, lds, stream); break;
      case 2: st = launch_frame<2>(a, nwg, lds, stream); break;
      default: st = launch_frame<1>(a, nwg, lds, stream); break;
    }
    if (st != TMCS_OK) return st;
  }
  if (overflow_out) return TMCS_OK;   // checked by the owner of the flag
  uint32_t hflag = 0;
  if ((st = hip_check(hipMemcpyAsync(&hflag, d->flag, sizeof(hflag), hipMemcpyDeviceToHost, stream), "flag copy")) != TMCS_OK)
    return st;
  if ((st = hip_check(hipStreamSynchronize(stream), "sample synchronize")) != TMCS_OK) return st;
  if (hflag) return fail(TMCS_EDEVICE, "noise event buffer overflow");
  return TMCS_OK;
}

tmcs_status sample_noalloc_run(const Circuit& c, uint64_t seed, uint32_t instance, uint64_t shot_begin,
                               uint64_t n_shots, uint64_t* det, uint64_t* obs, uint32_t* overflow, hipStream_t stream) {
  if (!overflow) return fail(TMCS_EINVAL, "null overflow flag");
  int dev = 0;
  tmcs_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st != TMCS_OK) return st;
  if (dev < 0 || dev >= 64) return fail(TMCS_EUNSUPPORTED, "device index beyond 63");
  const SampleDevice* d = (const SampleDevice*)c.device;
  if (!d || d->device != dev)
    return fail(TMCS_EINVAL, "the circuit's program is not on this device: call tmcs_sample or "
                             "tmcs_sample_async once on it first (the no-allocation call uploads nothing)");
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      if ((st = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress (scratch)")) != TMCS_OK)
        return st;
      g_scratch_ptr[dev] = (unsigned char*)ptr;
    }
    base = g_scratch_ptr[dev];
  }
  return sample_run(c, seed, instance, shot_begin, n_shots, det, obs, stream, nullptr, overflow,
                    const_cast<SampleDevice*>(d), base, NOALLOC_BYTES);
}

void* sample_state_new(const Circuit& c, tmcs_status* st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { *st = fail(TMCS_EDEVICE, "no HIP device"); return nullptr; }
  SampleDevice* d = nullptr;
  *st = build_state(c, dev, &d);
  return d;
}

void sample_state_free(void* state) {
  SampleDevice* d = (SampleDevice*)state;
  if (!d) return;
  free_device(d);
  delete d;
}

void sample_release(Circuit& c) {
  SampleDevice* d = (SampleDevice*)c.device;
  if (!d) return;
  free_device(d);
  delete d;
  c.device = nullptr;
}

}  // namespace tmcs
