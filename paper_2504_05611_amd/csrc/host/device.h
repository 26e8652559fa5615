// Entry points of the HIP side of the library (kernels and their launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace tmcs {

tmcs_status hip_check(hipError_t e, const char* what);

// sampler (sample.hip)
// blk_off (device, nullable): added to every block index of the noise streams;
// overflow_out (device, nullable): sticky event-buffer overflow flag owned by the
// caller, in which case the call neither clears nor checks it and never waits.
// fixed (device, nullable): event scratch of fixed_bytes bytes to use instead of
// the state's growing buffers (chunks are sized to fit it).
tmcs_status sample_run(const Circuit& c, uint64_t seed, uint32_t instance, uint64_t shot_begin,
                       uint64_t n_shots, uint64_t* det, uint64_t* obs, hipStream_t stream,
                       const uint64_t* blk_off = nullptr, uint32_t* overflow_out = nullptr,
                       void* state = nullptr, unsigned char* fixed = nullptr, size_t fixed_bytes = 0);
// tmcs_sample_noalloc: the sampler on the library's static device scratch; the
// circuit's program must already be on the current device.
tmcs_status sample_noalloc_run(const Circuit& c, uint64_t seed, uint32_t instance, uint64_t shot_begin,
                               uint64_t n_shots, uint64_t* det, uint64_t* obs, uint32_t* overflow,
                               hipStream_t stream);
// A private device state (program, tables, scratch) for callers whose launches
// must keep pointing at the same buffers, e.g. a captured graph; state = nullptr
// in sample_run uses the state cached on the circuit handle.
void* sample_state_new(const Circuit& c, tmcs_status* st);
void sample_state_free(void* state);
void sample_release(Circuit& c);

// decoder (decode.hip)
tmcs_status decode_run(const Dem& d, const tmcs_decoder_cfg& cfg, const uint64_t* det,
                       uint64_t n_shots, uint64_t* pred_obs, tmcs_decode_stats* stats,
                       hipStream_t stream, void* state = nullptr);
// Several decode items run as one batch (plans): staging per item, one BP launch
// per kernel variant and team size, one windowed-OSD launch.  Item buffers and
// states stay fixed, so the batch can be captured in a graph.
struct MultiItemSpec {
  const Dem* D;
  tmcs_decoder_cfg cfg;
  void* state;                 // decode_state_new
  const uint64_t* det;         // [rows][batch / 64]
  uint64_t* pred;              // [observables][batch / 64]
  tmcs_decode_stats* stats;    // device, may be null
};
struct MultiDecode;
tmcs_status decode_multi_create(const std::vector<MultiItemSpec>& items, uint64_t batch, hipStream_t stream,
                                MultiDecode** out);
tmcs_status decode_multi_enqueue(MultiDecode* m, hipStream_t stream);
void decode_multi_free(MultiDecode* m);
void* decode_state_new(const Dem& d, tmcs_status* st);
void decode_state_free(void* state);
tmcs_status ler_run(const uint64_t* pred, const uint64_t* obs, uint32_t k, uint64_t n_shots,
                    uint64_t* n_err, hipStream_t stream);
// adds the failing-shot count to a device counter (no wait)
tmcs_status count_errors_async(const uint64_t* pred, const uint64_t* obs, uint32_t k, uint64_t n_shots,
                               unsigned long long* counter, hipStream_t stream);
// launch-shape search for tmcs_autotune
tmcs_status autotune_run(const Dem& d, const uint64_t* det, uint64_t n_shots, tmcs_decoder_cfg* cfg,
                         hipStream_t stream);
void decode_release(Dem& d);

// circuit-distance search on the GPU (distance.hip)
tmcs_status dem_distance_device(const Dem& D, int max_active, int max_weight, int64_t max_states, int32_t* weight,
                                hipStream_t stream);

// weighted BP training kernels (wbp.hip)
size_t wbp_workspace_bytes(const Dem& d, int T, uint64_t n_shots);
tmcs_status wbp_forward_run(const Dem& d, const float* w, int T, const uint64_t* det,
                            uint64_t n_shots, float* llr, void* ws, size_t ws_bytes,
                            hipStream_t stream);
tmcs_status wbp_backward_run(const Dem& d, const float* w, int T, const uint64_t* det,
                             uint64_t n_shots, const float* gllr, float* gw, const void* ws,
                             size_t ws_bytes, hipStream_t stream);
void wbp_release(const Dem& d);
void wbp_set_global_state(bool on);

}  // namespace tmcs
