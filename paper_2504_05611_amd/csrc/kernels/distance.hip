// Circuit-level distance search on the GPU (Results, "Circuit-level distance of
// distributed primitives"; Table I lists upper bounds found by such searches).
//
// The same breadth-first search as the host version (host/distance.cpp), run
// level by level with one thread per state: level w holds the states (active
// detection events, observable mask) reachable with w mechanisms, and a state
// grows only by the mechanisms on its smallest active detector.  A state whose
// active set empties with a non-zero mask is a logical error of weight w.
// States whose active set exceeds max_active are dropped (an upper bound, as in
// Table I; exact when max_active covers every detector).
//
// Dedup: every state is entered once into a device hash table of 64-bit
// fingerprints of (active set, mask) (open addressing, linear probing, CAS).
// Two distinct states share a fingerprint with probability ~N^2 / 2^65 for N
// states (3e-4 at N = 1e8, 3e-8 at N = 1e6); such a collision drops a state,
// which can only make the search miss an error, never report a false one.
// The state budget is checked per level: the search stops, reporting nothing,
// when a level would push the total past max_states (the host version stops at
// the state that passes it), so the two agree whenever the budget suffices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../host/device.h"
#include "../host/timing.h"

namespace tmcs {

namespace {

constexpr int DCAP = 16;   // most active detection events a state can hold

struct DState {
  int32_t n;
  int32_t pad;
  uint64_t obs;
  int32_t d[DCAP];          // ascending; entries past n unused
};

struct DistArgs {
  const int32_t* row_ptr;   // CSR: detector -> columns
  const int32_t* col_idx;
  const int32_t* col_ptr;   // CSC: column -> detectors (ascending)
  const int32_t* row_idx;
  const uint64_t* obs;      // [cols]
  int32_t cols;
  int32_t cap;              // max_active
  uint64_t* table;          // [tmask + 1] fingerprints, 0 = empty
  uint64_t tmask;
  uint32_t max_probe;
  DState* next;             // appended states
  uint64_t next_cap;
  unsigned long long* counters;   // [0] next count, [1] found weight (min), [2] overflow
};

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  // splitmix64 finaliser
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

__device__ __forceinline__ uint64_t fingerprint(const int32_t* d, int n, uint64_t obs) {
  uint64_t h = mix64(obs ^ 0x9e3779b97f4a7c15ull * (uint64_t)(n + 1));
  for (int i = 0; i < n; ++i) h = mix64(h ^ ((uint64_t)(uint32_t)d[i] + 0x632be59bd9b4e019ull * (uint64_t)(i + 1)));
  return h ? h : 1ull;
}

// true when the fingerprint was not in the table (and is now)
__device__ __forceinline__ bool insert_new(const DistArgs& a, uint64_t fp) {
  uint64_t slot = fp & a.tmask;
  for (uint32_t p = 0; p < a.max_probe; ++p) {
    const unsigned long long prev = atomicCAS((unsigned long long*)&a.table[slot], 0ull, (unsigned long long)fp);
    if (prev == 0ull) return true;
    if (prev == fp) return false;
    slot = (slot + 1) & a.tmask;
  }
  atomicOr(&a.counters[2], 1ull);          // table too full: the search gives up
  return false;
}

__device__ __forceinline__ void emit(const DistArgs& a, const int32_t* d, int n, uint64_t obs, int w) {
  if (n == 0) {
    if (obs) atomicMin(&a.counters[1], (unsigned long long)w);
    return;
  }
  if (n > a.cap) return;
  if (!insert_new(a, fingerprint(d, n, obs))) return;
  const unsigned long long i = atomicAdd(&a.counters[0], 1ull);
  if (i >= a.next_cap) {
    atomicOr(&a.counters[2], 1ull);         // budget spent
    return;
  }
  DState& s = a.next[i];
  s.n = n;
  s.obs = obs;
  for (int k = 0; k < n; ++k) s.d[k] = d[k];
}

// Level 1: every mechanism on its own.
__global__ void k_dist_init(DistArgs a) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < a.cols; j += gridDim.x * blockDim.x) {
    const int b = a.col_ptr[j], n = a.col_ptr[j + 1] - b;
    if (n > a.cap) {
      continue;
    }
    int32_t d[DCAP];
    for (int k = 0; k < n; ++k) d[k] = a.row_idx[b + k];
    emit(a, d, n, a.obs[j], 1);
  }
}

// Level w: each state grows by the mechanisms on its smallest active detector
// (symmetric difference of two ascending lists).
__global__ void k_dist_expand(DistArgs a, const DState* cur, uint64_t ncur, int w) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncur; i += (uint64_t)gridDim.x * blockDim.x) {
    const DState s = cur[i];
    const int d0 = s.d[0];
    for (int32_t e = a.row_ptr[d0]; e < a.row_ptr[d0 + 1]; ++e) {
      const int j = a.col_idx[e];
      const int b = a.col_ptr[j], m = a.col_ptr[j + 1] - b;
      int32_t t[DCAP];
      int n = 0, x = 0, y = 0;
      bool over = false;
      while (x < s.n || y < m) {
        const int32_t u = x < s.n ? s.d[x] : 0x7fffffff;
        const int32_t v = y < m ? a.row_idx[b + y] : 0x7fffffff;
        int32_t out;
        if (u < v) { out = u; ++x; }
        else if (v < u) { out = v; ++y; }
        else { ++x; ++y; continue; }
        if (n == DCAP || n == a.cap) { over = true; break; }
        t[n++] = out;
      }
      if (over) continue;
      emit(a, t, n, s.obs ^ a.obs[j], w);
    }
  }
}

template <typename T>
tmcs_status upload_vec(T** dst, const std::vector<T>& v) {
  if (hipMalloc((void**)dst, std::max<size_t>(v.size(), 1) * sizeof(T)) != hipSuccess)
    return fail(TMCS_ENOMEM, "hipMalloc failed (distance search)");
  if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(TMCS_EDEVICE, "hipMemcpy failed (distance search)");
  return TMCS_OK;
}

__global__ void k_dist_counters(unsigned long long* c) {
  if (threadIdx.x < 4) c[threadIdx.x] = threadIdx.x == 1 ? 0xffffffffffffffffull : 0ull;
}

__global__ void k_dist_zero(unsigned long long* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

}  // namespace

tmcs_status dem_distance_device(const Dem& D, int max_active, int max_weight, int64_t max_states, int32_t* weight,
                                hipStream_t stream) {
  *weight = 0;
  if (D.obs_words != 1) return fail(TMCS_EUNSUPPORTED, "the distance search takes at most 64 observables");
  if (max_active < 1 || max_active > DCAP) return fail(TMCS_EINVAL, "max_active must be in [1, 16] on the device");
  if (max_weight < 1) return fail(TMCS_EINVAL, "max_weight must be positive");
  if (max_states < 1) return fail(TMCS_EINVAL, "max_states must be positive");
  DistArgs a{};
  std::vector<void*> owned;
  auto cleanup = [&]() { for (void* p : owned) hipFree(p); };
  int32_t *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr;
  uint64_t* ob = nullptr;
  tmcs_status st;
  st = upload_vec(&rp, D.row_ptr);
  owned.push_back(rp);
  if (st == TMCS_OK) { st = upload_vec(&ci, D.col_idx); owned.push_back(ci); }
  if (st == TMCS_OK) { st = upload_vec(&cp, D.col_ptr); owned.push_back(cp); }
  if (st == TMCS_OK) { st = upload_vec(&ri, D.row_idx); owned.push_back(ri); }
  if (st == TMCS_OK) { st = upload_vec(&ob, D.obs_mask); owned.push_back(ob); }
  if (st != TMCS_OK) {
    cleanup();
    return st;
  }
  // table: a power of two of at least twice the state budget
  uint64_t tsize = 1;
  while (tsize < 2 * (uint64_t)max_states) tsize <<= 1;
  uint64_t* table = nullptr;
  DState *lv0 = nullptr, *lv1 = nullptr;
  unsigned long long* ctr = nullptr;
  if (hipMalloc((void**)&table, tsize * sizeof(uint64_t)) != hipSuccess) { cleanup(); return fail(TMCS_ENOMEM, "hipMalloc failed (distance table)"); }
  owned.push_back(table);
  if (hipMalloc((void**)&lv0, (size_t)max_states * sizeof(DState)) != hipSuccess) { cleanup(); return fail(TMCS_ENOMEM, "hipMalloc failed (distance states)"); }
  owned.push_back(lv0);
  if (hipMalloc((void**)&lv1, (size_t)max_states * sizeof(DState)) != hipSuccess) { cleanup(); return fail(TMCS_ENOMEM, "hipMalloc failed (distance states)"); }
  owned.push_back(lv1);
  if (hipMalloc((void**)&ctr, 4 * sizeof(unsigned long long)) != hipSuccess) { cleanup(); return fail(TMCS_ENOMEM, "hipMalloc failed (distance counters)"); }
  owned.push_back(ctr);
  a.row_ptr = rp; a.col_idx = ci; a.col_ptr = cp; a.row_idx = ri; a.obs = ob; a.cols = D.cols; a.cap = max_active;
  a.table = table; a.tmask = tsize - 1; a.max_probe = 4096; a.counters = ctr;
  TMCS_LAUNCH("k_dist_zero", k_dist_zero, dim3(2048), dim3(256), 0, stream, (unsigned long long*)table, tsize);
  // counters: next count 0, smallest weight found = none, overflow 0
  const unsigned long long none = 0xffffffffffffffffull;
  TMCS_LAUNCH("k_dist_counters", k_dist_counters, dim3(1), dim3(64), 0, stream, ctr);
  uint64_t total = 0;
  DState* cur = lv0;
  DState* nxt = lv1;
  a.next = cur;
  a.next_cap = (uint64_t)max_states;
  TMCS_LAUNCH("k_dist_init", k_dist_init, dim3((unsigned)std::min<int64_t>((D.cols + 255) / 256, 4096)), dim3(256), 0,
              stream, a);
  for (int w = 1;; ++w) {
    unsigned long long h[4];
    if ((st = hip_check(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, stream), "distance counters")) != TMCS_OK ||
        (st = hip_check(hipStreamSynchronize(stream), "distance search")) != TMCS_OK) {
      cleanup();
      return st;
    }
    if (h[1] != none) { *weight = (int32_t)h[1]; break; }      // found at this level
    if (h[2]) break;                                            // budget or table spent: nothing found within it
    const uint64_t ncur = h[0];
    total += ncur;
    if (ncur == 0 || w >= max_weight) break;
    if (total >= (uint64_t)max_states) break;
    // expand the states just written (in a.next) into the other buffer; the
    // budget left bounds the next level
    cur = a.next;
    nxt = (cur == lv0) ? lv1 : lv0;
    a.next = nxt;
    a.next_cap = (uint64_t)max_states - total;
    TMCS_LAUNCH("k_dist_zero", k_dist_zero, dim3(1), dim3(64), 0, stream, ctr, (uint64_t)1);
    const int64_t grid = std::min<int64_t>((int64_t)((ncur + 255) / 256), 1 << 16);
    TMCS_LAUNCH("k_dist_expand", k_dist_expand, dim3((unsigned)grid), dim3(256), 0, stream, a, (const DState*)cur,
                (uint64_t)ncur, w + 1);
    if ((st = hip_check(hipGetLastError(), "k_dist_expand")) != TMCS_OK) { cleanup(); return st; }
  }
  cleanup();
  return TMCS_OK;
}

}  // namespace tmcs
