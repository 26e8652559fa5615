// Batch plans: preallocated sample -> decode -> count pipelines, optionally
// captured once into a HIP graph and replayed.
//
// A plan holds one or more items (a circuit, its DEM, decoder settings, a seed
// and an instance id).  Each replay processes the next batch of every item:
// shots [k*B, (k+1)*B) on the k-th replay, B a multiple of the 4096-shot noise
// block.  The absolute block index of the noise streams lives in device memory
// and is advanced by a kernel at the end of each replay, so one captured graph
// covers consecutive shot ranges and gives the same bits as eager calls on the
// same ranges.  Error counts, decoder statistics and the event-buffer overflow
// flag accumulate on the device and are read once by tmcs_plan_result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../host/device.h"
#include "../host/internal.h"
#include "../host/timing.h"

namespace tmcs {

namespace {

__global__ void k_advance(uint64_t* blk_off, uint64_t nblk) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *blk_off += nblk;
}

__global__ void k_fill_zero(uint64_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

struct Item {
  const Circuit* c = nullptr;
  const Dem* d = nullptr;
  tmcs_decoder_cfg cfg{};
  uint64_t seed = 0;
  uint32_t instance = 0;
  uint64_t* det = nullptr;
  uint64_t* obs = nullptr;
  uint64_t* pred = nullptr;
  // device block: [0] block offset, [1] errors, [2] overflow flag (u32), [3..] stats
  uint64_t* dev = nullptr;
  // private sampler / decoder states: a captured graph keeps pointing at their
  // scratch, which calls on the circuit and DEM handles may reallocate
  void* sstate = nullptr;
  void* dstate = nullptr;
};

}  // namespace

struct Plan {
  std::vector<Item> items;
  uint64_t batch = 0;
  uint64_t batches_done = 0;
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  // the items' samplers run side by side (a large circuit's frame kernel fills
  // a fraction of the GPU): one stream per item, forked from and joined back
  // to the plan's stream by events (branches of the captured graph)
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the items' decoders as one batch (one BP launch per kernel variant, one
  // windowed-OSD launch), or null when an item needs several decoder passes
  MultiDecode* multi = nullptr;
};

static constexpr int DEV_WORDS = 3 + (int)(sizeof(tmcs_decode_stats) / sizeof(uint64_t));

static tmcs_status enqueue_batch(Plan& p, hipStream_t s) {
  if (p.multi) {
    // sample every item (side by side), decode them together, then count
    tmcs_status st = hip_check(hipEventRecord(p.fork, s), "plan fork");
    for (size_t i = 0; i < p.items.size() && st == TMCS_OK; ++i) {
      Item& it = p.items[i];
      st = hip_check(hipStreamWaitEvent(p.side[i], p.fork, 0), "plan fork wait");
      if (st == TMCS_OK)
        st = sample_run(*it.c, it.seed, it.instance, 0, p.batch, it.det, it.obs, p.side[i], it.dev + 0,
                        (uint32_t*)(it.dev + 2), it.sstate);
      if (st == TMCS_OK) st = hip_check(hipEventRecord(p.join[i], p.side[i]), "plan join");
      if (st == TMCS_OK) st = hip_check(hipStreamWaitEvent(s, p.join[i], 0), "plan join wait");
    }
    if (st != TMCS_OK) return st;
    st = decode_multi_enqueue(p.multi, s);
    if (st != TMCS_OK) return st;
    for (Item& it : p.items) {
      st = count_errors_async(it.pred, it.obs, (uint32_t)it.c->num_obs, p.batch, (unsigned long long*)(it.dev + 1), s);
      if (st != TMCS_OK) return st;
      TMCS_LAUNCH("k_advance", k_advance, dim3(1), dim3(64), 0, s, it.dev + 0, (uint64_t)(p.batch / 4096));
      if ((st = hip_check(hipGetLastError(), "k_advance")) != TMCS_OK) return st;
    }
    return TMCS_OK;
  }
  for (Item& it : p.items) {
    tmcs_status st = sample_run(*it.c, it.seed, it.instance, 0, p.batch, it.det, it.obs, s, it.dev + 0,
                                (uint32_t*)(it.dev + 2), it.sstate);
    if (st != TMCS_OK) return st;
    st = decode_run(*it.d, it.cfg, it.det, p.batch, it.pred, (tmcs_decode_stats*)(it.dev + 3), s, it.dstate);
    if (st != TMCS_OK) return st;
    st = count_errors_async(it.pred, it.obs, (uint32_t)it.c->num_obs, p.batch, (unsigned long long*)(it.dev + 1), s);
    if (st != TMCS_OK) return st;
    TMCS_LAUNCH("k_advance", k_advance, dim3(1), dim3(64), 0, s, it.dev + 0, (uint64_t)(p.batch / 4096));
    if ((st = hip_check(hipGetLastError(), "k_advance")) != TMCS_OK) return st;
  }
  return TMCS_OK;
}

static void destroy(Plan* p) {
  if (!p) return;
  decode_multi_free(p->multi);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipStream_t x : p->side) (void)hipStreamDestroy(x);
  if (p->fork) (void)hipEventDestroy(p->fork);
  for (hipEvent_t e : p->join) (void)hipEventDestroy(e);
  for (Item& it : p->items) {
    sample_state_free(it.sstate);
    decode_state_free(it.dstate);
    hipFree(it.det);
    hipFree(it.obs);
    hipFree(it.pred);
    hipFree(it.dev);
  }
  delete p;
}

}  // namespace tmcs

struct tmcs_plan { tmcs::Plan* p; };

using namespace tmcs;

extern "C" {

tmcs_status tmcs_plan_create(const tmcs_plan_item* items, int32_t n_items, uint64_t batch_shots, int32_t use_graph,
                             tmcs_plan** out) {
  if (!items || n_items < 1 || !out) return fail(TMCS_EINVAL, "invalid plan arguments");
  if (batch_shots == 0 || batch_shots % 4096) return fail(TMCS_EINVAL, "batch_shots must be a positive multiple of 4096");
  *out = nullptr;
  Plan* p = new (std::nothrow) Plan();
  if (!p) return fail(TMCS_ENOMEM, "host allocation failed");
  // no timing events in the warm-up batch or the captured graph
  struct TimingOff {
    bool was = timing_on();
    TimingOff() { if (was) tmcs_timing_enable(0); }
    ~TimingOff() { if (was) tmcs_timing_enable(1); }
  } timing_off;
  p->batch = batch_shots;
  p->use_graph = use_graph != 0;
  const int64_t words = (int64_t)(batch_shots / 64);
  tmcs_status st = TMCS_OK;
  for (int i = 0; i < n_items && st == TMCS_OK; ++i) {
    const tmcs_plan_item& in = items[i];
    if (!in.circuit || !in.dem) { st = fail(TMCS_EINVAL, "plan item without circuit or DEM"); break; }
    if (in.cfg.ehat_dev || in.cfg.llr_dev || in.cfg.iters_dev || in.cfg.flags_dev) {
      st = fail(TMCS_EINVAL, "plans do not take per-shot decoder outputs");
      break;
    }
    Item it;
    it.c = &in.circuit->c;
    it.d = &in.dem->d;
    it.cfg = in.cfg;
    it.seed = in.seed;
    it.instance = in.instance;
    if (it.d->rows != it.c->num_dets || it.d->nobs != it.c->num_obs) {
      st = fail(TMCS_EINVAL, "plan item: DEM does not belong to the circuit");
      break;
    }
    const size_t dbytes = (size_t)std::max(it.c->num_dets, 1) * words * 8;
    const size_t obytes = (size_t)std::max(it.c->num_obs, 1) * words * 8;
    if (hipMalloc((void**)&it.det, dbytes) != hipSuccess || hipMalloc((void**)&it.obs, obytes) != hipSuccess ||
        hipMalloc((void**)&it.pred, obytes) != hipSuccess ||
        hipMalloc((void**)&it.dev, DEV_WORDS * sizeof(uint64_t)) != hipSuccess) {
      p->items.push_back(it);
      st = fail(TMCS_ENOMEM, "hipMalloc failed (plan buffers)");
      break;
    }
    it.sstate = sample_state_new(*it.c, &st);
    if (st == TMCS_OK) it.dstate = decode_state_new(*it.d, &st);
    p->items.push_back(it);
  }
  if (st == TMCS_OK) st = hip_check(hipStreamCreate(&p->cap_stream), "hipStreamCreate");
  if (st == TMCS_OK) st = hip_check(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming), "hipEventCreate");
  for (size_t i = 0; i < p->items.size() && st == TMCS_OK; ++i) {
    hipStream_t x = nullptr;
    hipEvent_t e = nullptr;
    st = hip_check(hipStreamCreate(&x), "hipStreamCreate");
    if (st == TMCS_OK) p->side.push_back(x);
    if (st == TMCS_OK) st = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    if (st == TMCS_OK) p->join.push_back(e);
  }
  if (st == TMCS_OK) {
    std::vector<MultiItemSpec> specs;
    for (Item& it : p->items)
      specs.push_back(MultiItemSpec{it.d, it.cfg, it.dstate, it.det, it.pred, (tmcs_decode_stats*)(it.dev + 3)});
    const tmcs_status sm = decode_multi_create(specs, batch_shots, p->cap_stream, &p->multi);
    if (sm == TMCS_EUNSUPPORTED) p->multi = nullptr;        // items decode one after another
    else st = sm;
  }
  if (st == TMCS_OK) {
    // one eager batch allocates every scratch buffer, then the counters are reset
    for (Item& it : p->items)
      TMCS_LAUNCH("k_fill_zero", k_fill_zero, dim3((DEV_WORDS + 63) / 64), dim3(64), 0, p->cap_stream, it.dev, DEV_WORDS);
    st = enqueue_batch(*p, p->cap_stream);
    if (st == TMCS_OK) st = hip_check(hipStreamSynchronize(p->cap_stream), "plan warm-up");
    for (Item& it : p->items)
      TMCS_LAUNCH("k_fill_zero", k_fill_zero, dim3((DEV_WORDS + 63) / 64), dim3(64), 0, p->cap_stream, it.dev, DEV_WORDS);
    if (st == TMCS_OK) st = hip_check(hipStreamSynchronize(p->cap_stream), "plan reset");
  }
  if (st == TMCS_OK && p->use_graph) {
    st = hip_check(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (st == TMCS_OK) {
      tmcs_status st2 = enqueue_batch(*p, p->cap_stream);
      hipGraph_t g = nullptr;
      st = hip_check(hipStreamEndCapture(p->cap_stream, &g), "hipStreamEndCapture");
      p->graph = g;
      if (st == TMCS_OK) st = st2;
    }
    if (st == TMCS_OK)
      st = hip_check(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  }
  if (st != TMCS_OK) {
    destroy(p);
    return st;
  }
  tmcs_plan* h = new (std::nothrow) tmcs_plan{p};
  if (!h) { destroy(p); return fail(TMCS_ENOMEM, "host allocation failed"); }
  *out = h;
  return TMCS_OK;
}

tmcs_status tmcs_plan_run(tmcs_plan* h, uint32_t n_batches, void* stream) {
  if (!h) return fail(TMCS_EINVAL, "null plan");
  Plan& p = *h->p;
  hipStream_t s = (hipStream_t)stream;
  for (uint32_t b = 0; b < n_batches; ++b) {
    tmcs_status st;
    // with kernel timing on, the batch runs as eager launches of the same
    // kernels on the same buffers, so that each launch is timed
    if (p.use_graph && !timing_on()) st = hip_check(hipGraphLaunch(p.exec, s), "hipGraphLaunch");
    else st = enqueue_batch(p, s);
    if (st != TMCS_OK) return st;
    ++p.batches_done;
  }
  return TMCS_OK;
}

tmcs_status tmcs_plan_result(tmcs_plan* h, int32_t item, uint64_t* shots, uint64_t* errors,
                             tmcs_decode_stats* stats, void* stream) {
  if (!h) return fail(TMCS_EINVAL, "null plan");
  Plan& p = *h->p;
  if (item < 0 || item >= (int32_t)p.items.size()) return fail(TMCS_EINVAL, "plan item out of range");
  uint64_t host[DEV_WORDS];
  tmcs_status st = hip_check(hipMemcpyAsync(host, p.items[item].dev, sizeof(host), hipMemcpyDeviceToHost,
                                            (hipStream_t)stream), "plan result copy");
  if (st == TMCS_OK) st = hip_check(hipStreamSynchronize((hipStream_t)stream), "plan result");
  if (st != TMCS_OK) return st;
  if ((uint32_t)host[2]) return fail(TMCS_EDEVICE, "noise event buffer overflow during the plan");
  if (shots) *shots = p.batches_done * p.batch;
  if (errors) *errors = host[1];
  if (stats) std::memcpy(stats, host + 3, sizeof(tmcs_decode_stats));
  return TMCS_OK;
}

void tmcs_plan_free(tmcs_plan* h) {
  if (!h) return;
  destroy(h->p);
  delete h;
}

tmcs_status tmcs_autotune(const tmcs_dem* d, const uint64_t* det_dev, uint64_t n_shots, tmcs_decoder_cfg* cfg,
                          void* stream) {
  if (!d || !det_dev || !cfg) return fail(TMCS_EINVAL, "null argument");
  return autotune_run(d->d, det_dev, n_shots, cfg, (hipStream_t)stream);
}

}  // extern "C"
