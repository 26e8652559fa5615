// C ABI of the library: argument validation, handle ownership and errors.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "device.h"
#include "internal.h"

namespace tmcs {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

tmcs_status fail(tmcs_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

tmcs_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return TMCS_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? TMCS_ENOMEM : TMCS_EDEVICE;
}

}  // namespace tmcs

using namespace tmcs;

#define TMCS_TRY(body)                                               \
  try {                                                              \
    body                                                             \
  } catch (const std::bad_alloc&) {                                  \
    return fail(TMCS_ENOMEM, "host allocation failed");              \
  } catch (const std::exception& ex) {                               \
    return fail(TMCS_EINVAL, std::string("exception: ") + ex.what()); \
  }

extern "C" {

tmcs_status tmcs_build_circuit(const tmcs_circuit_spec* spec, tmcs_circuit** out) {
  if (!spec || !out) return fail(TMCS_EINVAL, "null argument");
  *out = nullptr;
  TMCS_TRY({
    tmcs_circuit* h = new tmcs_circuit();
    tmcs_status st = build_circuit(*spec, &h->c);
    if (st != TMCS_OK) { delete h; return st; }
    *out = h;
    set_error("");
    return TMCS_OK;
  })
}

void tmcs_free_circuit(tmcs_circuit* c) {
  if (!c) return;
  sample_release(c->c);
  delete c;
}

tmcs_status tmcs_circuit_info(const tmcs_circuit* c, int64_t info[TMCS_INFO_LEN]) {
  if (!c || !info) return fail(TMCS_EINVAL, "null argument");
  circuit_counts(c->c, info);
  return TMCS_OK;
}

tmcs_status tmcs_circuit_text(const tmcs_circuit* c, char* buf, size_t cap, size_t* len) {
  if (!c) return fail(TMCS_EINVAL, "null circuit");
  TMCS_TRY({
    const std::string s = circuit_text(c->c);
    if (len) *len = s.size();
    if (buf && cap) {
      const size_t n = s.size() < cap - 1 ? s.size() : cap - 1;
      std::memcpy(buf, s.data(), n);
      buf[n] = '\0';
    }
    return TMCS_OK;
  })
}

tmcs_status tmcs_build_dem(const tmcs_circuit* c, tmcs_dem** out) {
  if (!c || !out) return fail(TMCS_EINVAL, "null argument");
  *out = nullptr;
  TMCS_TRY({
    tmcs_dem* h = new tmcs_dem();
    tmcs_status st = build_dem(c->c, &h->d);
    if (st != TMCS_OK) { delete h; return st; }
    *out = h;
    return TMCS_OK;
  })
}

void tmcs_free_dem(tmcs_dem* d) {
  if (!d) return;
  decode_release(d->d);
  wbp_release(d->d);
  delete d;
}

tmcs_status tmcs_dem_info(const tmcs_dem* d, int64_t info[TMCS_DEM_INFO_LEN]) {
  if (!d || !info) return fail(TMCS_EINVAL, "null argument");
  for (int i = 0; i < TMCS_DEM_INFO_LEN; ++i) info[i] = 0;
  info[TMCS_DEM_ROWS] = d->d.rows;
  info[TMCS_DEM_COLS] = d->d.cols;
  info[TMCS_DEM_OBS] = d->d.nobs;
  info[TMCS_DEM_EDGES] = d->d.edges;
  info[TMCS_DEM_RANK] = d->d.rank;
  info[TMCS_DEM_UNDETECTABLE] = d->d.undetectable;
  info[TMCS_DEM_MAX_ROW_DEG] = d->d.max_row_deg;
  info[TMCS_DEM_MAX_COL_DEG] = d->d.max_col_deg;
  return TMCS_OK;
}

tmcs_status tmcs_dem_distance(const tmcs_dem* d, int32_t max_active, int32_t max_weight, int64_t max_states,
                              int32_t* weight) {
  if (!d || !weight || max_active < 1 || max_weight < 1 || max_states < 1) return fail(TMCS_EINVAL, "invalid argument");
  TMCS_TRY({ return dem_distance(d->d, max_active, max_weight, max_states, weight); })
}

tmcs_status tmcs_dem_distance_device(const tmcs_dem* d, int32_t max_active, int32_t max_weight, int64_t max_states,
                                     int32_t* weight, void* stream) {
  if (!d || !weight) return fail(TMCS_EINVAL, "invalid argument");
  TMCS_TRY({ return dem_distance_device(d->d, max_active, max_weight, max_states, weight, (hipStream_t)stream); })
}

tmcs_status tmcs_dem_export(const tmcs_dem* d, int32_t* col_ptr, int32_t* row_idx, double* priors,
                            uint64_t* obs_mask) {
  if (!d) return fail(TMCS_EINVAL, "null dem");
  const Dem& D = d->d;
  if (col_ptr) std::memcpy(col_ptr, D.col_ptr.data(), D.col_ptr.size() * sizeof(int32_t));
  if (row_idx && D.edges) std::memcpy(row_idx, D.row_idx.data(), D.row_idx.size() * sizeof(int32_t));
  if (priors && D.cols) std::memcpy(priors, D.priors.data(), D.priors.size() * sizeof(double));
  if (obs_mask && D.cols) std::memcpy(obs_mask, D.obs_mask.data(), D.obs_mask.size() * sizeof(uint64_t));
  return TMCS_OK;
}

tmcs_status tmcs_sample(const tmcs_circuit* c, uint64_t seed, uint32_t instance, uint64_t shot_begin,
                        uint64_t n_shots, uint64_t* det_dev, uint64_t* obs_dev, void* stream) {
  if (!c) return fail(TMCS_EINVAL, "null circuit");
  TMCS_TRY({
    return sample_run(c->c, seed, instance, shot_begin, n_shots, det_dev, obs_dev, (hipStream_t)stream);
  })
}

tmcs_status tmcs_sample_async(const tmcs_circuit* c, uint64_t seed, uint32_t instance, uint64_t shot_begin,
                              uint64_t n_shots, uint64_t* det_dev, uint64_t* obs_dev, uint32_t* overflow_dev,
                              void* stream) {
  if (!c) return fail(TMCS_EINVAL, "null circuit");
  if (!overflow_dev) return fail(TMCS_EINVAL, "null overflow flag");
  TMCS_TRY({
    return sample_run(c->c, seed, instance, shot_begin, n_shots, det_dev, obs_dev, (hipStream_t)stream, nullptr,
                      overflow_dev);
  })
}

tmcs_status tmcs_sample_noalloc(const tmcs_circuit* c, uint64_t seed, uint32_t instance, uint64_t shot_begin,
                                uint64_t n_shots, uint64_t* det_dev, uint64_t* obs_dev, uint32_t* overflow_dev,
                                void* stream) {
  if (!c) return fail(TMCS_EINVAL, "null circuit");
  TMCS_TRY({
    return sample_noalloc_run(c->c, seed, instance, shot_begin, n_shots, det_dev, obs_dev, overflow_dev,
                              (hipStream_t)stream);
  })
}

tmcs_status tmcs_decode(const tmcs_dem* d, const tmcs_decoder_cfg* cfg, const uint64_t* det_dev,
                        uint64_t n_shots, uint64_t* pred_obs_dev, tmcs_decode_stats* stats_dev,
                        void* stream) {
  if (!d || !cfg) return fail(TMCS_EINVAL, "null argument");
  if (cfg->max_iter < 1 || cfg->max_iter > 100000) return fail(TMCS_EINVAL, "max_iter must be in [1, 100000]");
  if (!std::isfinite(cfg->alpha) || cfg->alpha <= 0.0f) return fail(TMCS_EINVAL, "alpha must be positive");
  if (cfg->osd_window < 0 || cfg->osd_window > 2048) return fail(TMCS_EINVAL, "osd_window must be in [0, 2048]");
  if (cfg->osd_order < 0 || cfg->osd_order > 64) return fail(TMCS_EINVAL, "osd_order must be in [0, 64]");
  if (cfg->decode_chunk < 0 || cfg->decode_chunk % 64 != 0)
    return fail(TMCS_EINVAL, "decode_chunk must be 0 or a positive multiple of 64");
  if (cfg->bp_sched < 0 || cfg->bp_sched > 2) return fail(TMCS_EINVAL, "bp_sched must be 0, 1 or 2");
  if (cfg->bp_global_state < 0 || cfg->bp_global_state > 3)
    return fail(TMCS_EINVAL, "bp_global_state must be 0, 1, 2 or 3");
  TMCS_TRY({
    return decode_run(d->d, *cfg, det_dev, n_shots, pred_obs_dev, stats_dev, (hipStream_t)stream);
  })
}

tmcs_status tmcs_count_errors(const uint64_t* pred_obs_dev, const uint64_t* obs_dev, uint32_t k, uint64_t n_shots,
                              uint64_t* n_errors_dev, void* stream) {
  if (!n_errors_dev) return fail(TMCS_EINVAL, "null error counter");
  TMCS_TRY({
    return count_errors_async(pred_obs_dev, obs_dev, k, n_shots, (unsigned long long*)n_errors_dev,
                              (hipStream_t)stream);
  })
}

tmcs_status tmcs_logical_error_rate(const uint64_t* pred_obs_dev, const uint64_t* obs_dev, uint32_t k,
                                    uint64_t n_shots, uint64_t* n_errors_host, double* ler, double* sigma,
                                    void* stream) {
  uint64_t ne = 0;
  TMCS_TRY({
    tmcs_status st = ler_run(pred_obs_dev, obs_dev, k, n_shots, &ne, (hipStream_t)stream);
    if (st != TMCS_OK) return st;
    const double p = n_shots ? (double)ne / (double)n_shots : 0.0;
    if (n_errors_host) *n_errors_host = ne;
    if (ler) *ler = p;
    if (sigma) *sigma = n_shots ? std::sqrt(p * (1.0 - p) / (double)n_shots) : 0.0;
    return TMCS_OK;
  })
}

tmcs_status tmcs_wbp_global_state(int32_t on) {
  wbp_set_global_state(on != 0);
  return TMCS_OK;
}

tmcs_status tmcs_wbp_workspace_size(const tmcs_dem* d, int32_t T, uint64_t n_shots, size_t* bytes) {
  if (!d || !bytes || T < 1) return fail(TMCS_EINVAL, "invalid argument");
  *bytes = wbp_workspace_bytes(d->d, T, n_shots);
  return TMCS_OK;
}

tmcs_status tmcs_wbp_forward(const tmcs_dem* d, const float* weights_dev, int32_t T, const uint64_t* det_dev,
                             uint64_t n_shots, float* llr_dev, void* workspace_dev, size_t workspace_bytes,
                             void* stream) {
  if (!d || !weights_dev || T < 1) return fail(TMCS_EINVAL, "invalid argument");
  TMCS_TRY({
    return wbp_forward_run(d->d, weights_dev, T, det_dev, n_shots, llr_dev, workspace_dev, workspace_bytes,
                           (hipStream_t)stream);
  })
}

tmcs_status tmcs_wbp_backward(const tmcs_dem* d, const float* weights_dev, int32_t T, const uint64_t* det_dev,
                              uint64_t n_shots, const float* grad_llr_dev, float* grad_w_dev,
                              const void* workspace_dev, size_t workspace_bytes, void* stream) {
  if (!d || !weights_dev || !grad_llr_dev || !grad_w_dev || T < 1) return fail(TMCS_EINVAL, "invalid argument");
  TMCS_TRY({
    return wbp_backward_run(d->d, weights_dev, T, det_dev, n_shots, grad_llr_dev, grad_w_dev, workspace_dev,
                            workspace_bytes, (hipStream_t)stream);
  })
}

const char* tmcs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
