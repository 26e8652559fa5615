// Entry points of the HIP side of the library (kernels and their launchers).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tmcs {

tmcs_status hip_check(hipError_t e, const char* what);

// sampler (sample.hip)
tmcs_status sample_run(const Circuit& c, uint64_t seed, uint32_t instance, uint64_t shot_begin,
                       uint64_t n_shots, uint64_t* det, uint64_t* obs, hipStream_t stream);
void sample_release(Circuit& c);

// decoder (decode.hip)
tmcs_status decode_run(const Dem& d, const tmcs_decoder_cfg& cfg, const uint64_t* det,
                       uint64_t n_shots, uint64_t* pred_obs, tmcs_decode_stats* stats,
                       hipStream_t stream);
tmcs_status ler_run(const uint64_t* pred, const uint64_t* obs, uint32_t k, uint64_t n_shots,
                    uint64_t* n_err, hipStream_t stream);
void decode_release(Dem& d);

// weighted BP training kernels (wbp.hip)
size_t wbp_workspace_bytes(const Dem& d, int T, uint64_t n_shots);
tmcs_status wbp_forward_run(const Dem& d, const float* w, int T, const uint64_t* det,
                            uint64_t n_shots, float* llr, void* ws, size_t ws_bytes,
                            hipStream_t stream);
tmcs_status wbp_backward_run(const Dem& d, const float* w, int T, const uint64_t* det,
                             uint64_t n_shots, const float* gllr, float* gw, const void* ws,
                             size_t ws_bytes, hipStream_t stream);
void wbp_release(const Dem& d);

}  // namespace tmcs
