/*
 * tmcs.h - C ABI of the MI355X Monte-Carlo shot pipeline for distributed
 * transversal QEC operations (non-local transversal CNOT and logical
 * teleportation over ebit layers, on rotated surface codes and
 * bivariate-bicycle codes).
 *
 * The pipeline follows the paper's statement of the problem (Methods,
 * "Simulation" and "Decoding"): build a noisy Clifford circuit for the
 * operation, extract its detector error model (DEM) - a parity-check matrix
 * whose rows are detectors and whose columns are distinct error mechanisms -
 * sample detector and observable bits shot by shot, decode each syndrome, and
 * count the shots in which any logical observable is wrong (the whole-operation
 * logical error rate).
 *
 * Conventions
 *  - Every call returns a tmcs_status and never aborts; tmcs_last_error()
 *    returns a thread-local message describing the last failure.
 *  - Handles (tmcs_circuit, tmcs_dem) are owned by the library and released
 *    with tmcs_free_*.  All other buffers are owned by the caller.
 *  - "_dev" pointers are device (HBM) pointers on the current HIP device;
 *    "stream" is a hipStream_t passed as void* (NULL = default stream).
 *    Device work is enqueued on that stream and returns without waiting,
 *    except where a function says it synchronises.
 *  - Bit-packed shot arrays are row-major [rows][ceil(n_shots/64)] uint64:
 *    shot i of the call is bit (i % 64) of word (i / 64), least significant
 *    bit first.  Bits past n_shots in the last word are written as 0.
 *  - Outputs are pure functions of (spec, seed, instance, shot range): they
 *    do not depend on launch shapes, tile sizes or the order of calls.
 */
#ifndef TMCS_H
#define TMCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TMCS_OK = 0,
  TMCS_EINVAL = 1,            /* invalid argument (message says which) */
  TMCS_ENOMEM = 2,            /* host or device allocation failed */
  TMCS_EDEVICE = 3,           /* a HIP call failed (possibly an earlier async fault) */
  TMCS_EUNSUPPORTED = 4,      /* valid request outside what this build supports */
  TMCS_ENONDETERMINISTIC = 5  /* tmcs_build_dem: a detector or observable is random in the
                                 noiseless circuit (the message names it) */
} tmcs_status;

enum { TMCS_SC = 0, TMCS_BB = 1 };                                  /* code family */
enum { TMCS_MEMORY = 0, TMCS_NONLOCAL_CNOT = 1, TMCS_TELEPORT = 2, TMCS_PAULI_STRING = 3 }; /* operation */

/* Circuit specification.
 *  Rotated surface code [[d^2,1,d]] (Supplementary Note 2): code = TMCS_SC, d odd >= 3.
 *  Bivariate-bicycle code (Supplementary Note 3, Table IV): code = TMCS_BB with
 *  x = S_l (x) I_m, y = I_l (x) S_m, a(x,y) = sum_k x^bb_a[k][0] y^bb_a[k][1],
 *  b(x,y) likewise; H_X = [A|B], H_Z = [B^T|A^T].
 *  op: TMCS_MEMORY (rounds_before rounds, rounds_after ignored),
 *      TMCS_NONLOCAL_CNOT (Methods, "Non-local CNOT circuit"; Fig. 1b),
 *      TMCS_TELEPORT (Methods, "State teleportation circuit"; Fig. 1c);
 *      the paper's runs use rounds_before = 4, rounds_after = 3.
 *  p: circuit-level error rate (reset/measurement flips, gate depolarizing,
 *     BB idle depolarizing); p_ebit: 2-qubit depolarizing on each ebit pair
 *     (Methods, "Simulation").  0 <= p, p_ebit < 0.5.
 */
typedef struct {
  int32_t code;
  int32_t d;
  int32_t bb_l, bb_m;
  int32_t bb_a[3][2];
  int32_t bb_b[3][2];
  int32_t op;
  int32_t rounds_before, rounds_after;
  double p, p_ebit;
  /* ebit decoherence (Methods, Decoherence; T1 = T2 = T): the n ebits of a
   * non-local CNOT are made ebit_per_step at a time (0: no decoherence), the last
   * group just before the CNOT, so ebit k has waited
   * age_k = ceil(n / ebit_per_step) - 1 - floor(k / ebit_per_step) generation
   * steps.  Both halves then get DEPOLARIZE1(3/4 (1 - exp(-age_k * ebit_rate)))
   * (p_X = p_Y = p_Z = (1 - exp(-t/T)) / 4), with ebit_rate = t_gen / T. */
  int32_t ebit_per_step;
  double ebit_rate;
  /* TMCS_PAULI_STRING (Methods, "Pauli string compute"): weight w >= 2 data blocks
   * and one ancilla block, rounds_before rounds on all of them, then the chain of
   * block CNOTs 1 -> 2 -> ... -> w (non-local for the 1st, 3rd, ... link, local
   * transversal for the others) and a local CNOT w -> ancilla, each followed by
   * one round on its two blocks; every block's Z logicals are observables (at
   * most 256 in all).  rounds_after is ignored. */
  int32_t weight;
} tmcs_circuit_spec;

typedef struct tmcs_circuit tmcs_circuit; /* opaque, library-owned */
typedef struct tmcs_dem tmcs_dem;         /* opaque, library-owned */

/* Indices into the info arrays. */
enum {
  TMCS_INFO_QUBITS = 0, TMCS_INFO_GATES_1Q, TMCS_INFO_GATES_2Q, TMCS_INFO_MEAS,
  TMCS_INFO_MEAS_FINAL, TMCS_INFO_DETECTORS, TMCS_INFO_OBSERVABLES,
  TMCS_INFO_NOISE_SITES, TMCS_INFO_INSTRUCTIONS, TMCS_INFO_CODE_N, TMCS_INFO_CODE_K,
  TMCS_INFO_EVENTS_PER_MSHOT,   /* expected noise events per 10^6 shots (sum of site p), rounded */
  TMCS_INFO_LEN = 16
};
enum {
  TMCS_DEM_ROWS = 0, TMCS_DEM_COLS, TMCS_DEM_OBS, TMCS_DEM_EDGES, TMCS_DEM_RANK,
  TMCS_DEM_UNDETECTABLE, TMCS_DEM_MAX_ROW_DEG, TMCS_DEM_MAX_COL_DEG,
  TMCS_DEM_INFO_LEN = 16
};

/* Build the noisy circuit of an operation (host only, no device work).
 * Noise model and schedules: Methods "Simulation"; Table III fixes the gate
 * and measurement counts the builder reproduces.  *out receives a new handle. */
tmcs_status tmcs_build_circuit(const tmcs_circuit_spec* spec, tmcs_circuit** out);
void tmcs_free_circuit(tmcs_circuit* c);

/* Counts (Table III style): info[TMCS_INFO_*]; TMCS_INFO_MEAS includes the final
 * data readout, TMCS_INFO_MEAS_FINAL is that readout alone. */
tmcs_status tmcs_circuit_info(const tmcs_circuit* c, int64_t info[TMCS_INFO_LEN]);

/* Canonical text of the circuit (stim-like syntax, relative record indices).
 * Writes at most cap bytes including the terminating NUL; *len receives the
 * full length without NUL (call with buf = NULL, cap = 0 to size the buffer). */
tmcs_status tmcs_circuit_text(const tmcs_circuit* c, char* buf, size_t cap, size_t* len);

/* Detector error model (Methods, "Decoding"): every single fault of every noise
 * site is propagated to the detectors and observables it flips (a backward
 * sensitivity sweep over the circuit); identical symptoms are merged with
 * p <- pa + pb - 2 pa pb in circuit order; columns are sorted by (detector
 * list, observable mask).  Host only; device copies are made on first use.
 * The same sweep checks that every detector and observable has a fixed value
 * in the noiseless circuit (detectors compare stabilizer measurements, Methods
 * "Simulation"); otherwise the call fails with TMCS_ENONDETERMINISTIC. */
tmcs_status tmcs_build_dem(const tmcs_circuit* c, tmcs_dem** out);
void tmcs_free_dem(tmcs_dem* d);
tmcs_status tmcs_dem_info(const tmcs_dem* d, int64_t info[TMCS_DEM_INFO_LEN]);

/* Host copy of the DEM: column-compressed H (col_ptr[cols+1], row_idx[edges],
 * rows ascending within a column), priors[cols], obs_mask[cols][ceil(obs/64)]
 * (bit o % 64 of word o / 64 set when the mechanism flips observable o; one
 * word per column up to 64 observables, at most 256 observables).  Columns are
 * sorted by detector list, then by the mask read as one integer.  NULL
 * pointers skip. */
tmcs_status tmcs_dem_export(const tmcs_dem* d, int32_t* col_ptr, int32_t* row_idx,
                            double* priors, uint64_t* obs_mask);

/* Circuit-level distance search (Results, "Circuit-level distance of distributed
 * primitives"; Table I lists upper bounds): *weight receives the fewest DEM
 * mechanisms found whose detector flips cancel while an observable flips, or 0
 * when none is found with at most max_weight mechanisms, intermediate sets of
 * at most max_active detection events and at most max_states search states.
 * Breadth-first over (active detection events, observable mask), growing a state
 * only by mechanisms on its smallest active detector; exact when max_active is
 * at least the number of detectors and the state budget suffices, an upper
 * bound otherwise.  Host only; DEMs with at most 64 observables. */
tmcs_status tmcs_dem_distance(const tmcs_dem* d, int32_t max_active, int32_t max_weight,
                              int64_t max_states, int32_t* weight);

/* The same search on the GPU, level by level with one thread per state and the
 * visited states in a device hash table of 64-bit fingerprints (two distinct
 * states collide with probability ~N^2 / 2^65 for N states; a collision can
 * only hide an error, never report a false one).  max_active <= 16.  The state
 * budget is checked per level (a level that would pass max_states ends the
 * search with *weight = 0); with a sufficient budget the result equals
 * tmcs_dem_distance's.  Allocates about 80 * 2 * max_states bytes of states and
 * 16 * max_states bytes of table for the call; synchronises the stream. */
tmcs_status tmcs_dem_distance_device(const tmcs_dem* d, int32_t max_active, int32_t max_weight,
                                     int64_t max_states, int32_t* weight, void* stream);

/* Sample n_shots shots [shot_begin, shot_begin + n_shots) of circuit c.
 * Noise: Philox4x32-10 with key (seed lo, seed hi) and counter (block, site,
 * instance, call) draws the events of each noise site per 4096-shot block; a draw
 * u gives g = #{k in 1..4096 : u < ceil((1-p)^k 2^32)} event-free shots before
 * the next event, and a K-component channel picks component (v K) >> 32 from the
 * next draw v.  shot_begin must be a multiple of 64.
 * det_dev: [detectors][ceil(n/64)] uint64; obs_dev: [observables][ceil(n/64)].
 * Scratch device memory is cached on the circuit handle and grows on demand;
 * the call synchronises the stream once to check the event-buffer capacity. */
tmcs_status tmcs_sample(const tmcs_circuit* c, uint64_t seed, uint32_t instance,
                        uint64_t shot_begin, uint64_t n_shots, uint64_t* det_dev,
                        uint64_t* obs_dev, void* stream);

/* tmcs_sample without the wait, for pipelines that keep the device busy: the
 * same shots and outputs, but an event-buffer overflow sets *overflow_dev
 * (device uint32 that the caller zeroes; it stays set) instead of returning an
 * error, and the call never synchronises.  The caller checks the flag after the
 * work; outputs of calls made while it was set are not valid.  NULL
 * overflow_dev: TMCS_EINVAL. */
tmcs_status tmcs_sample_async(const tmcs_circuit* c, uint64_t seed, uint32_t instance,
                              uint64_t shot_begin, uint64_t n_shots, uint64_t* det_dev,
                              uint64_t* obs_dev, uint32_t* overflow_dev, void* stream);

/* tmcs_sample_async for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * shots and outputs, but the event scratch (per-(block, site) counts and offsets,
 * scan partials, the event buffer) lives in a fixed 64 MiB device array of the
 * library, one per GPU, held until the process ends; the call allocates nothing
 * and never waits.  Shot ranges are processed in chunks of 4096-shot blocks that
 * fit that array.  Requirements and errors:
 *  - the circuit's program must already be on the current device (any earlier
 *    tmcs_sample / tmcs_sample_async call there uploads it); otherwise TMCS_EINVAL;
 *  - overflow_dev as for tmcs_sample_async (NULL: TMCS_EINVAL);
 *  - a circuit whose event scratch for one 4096-shot block exceeds 64 MiB
 *    (roughly > 1.5e3 expected noise events per shot): TMCS_EUNSUPPORTED.
 * All calls on one GPU share the array, which keeps the last call's contents
 * (every call overwrites what it reads): calls that overlap in time on one GPU
 * (different streams, or several host threads) race and give invalid outputs. */
tmcs_status tmcs_sample_noalloc(const tmcs_circuit* c, uint64_t seed, uint32_t instance,
                                uint64_t shot_begin, uint64_t n_shots, uint64_t* det_dev,
                                uint64_t* obs_dev, uint32_t* overflow_dev, void* stream);

/* Decoder configuration: flooding min-sum BP over the DEM with an OSD-0 fallback
 * (Supplementary Note 7 names BP-OSD).  With priors lambda_v = ln((1-p_v)/p_v):
 *   m_{c->v} = (-1)^{s_c} prod_{v' != v} sgn(q_{v'->c}) * alpha * min_{v' != v} |q_{v'->c}|,
 *   L_v = lambda_v + sum_c m_{c->v} (c ascending), q_{v->c} = L_v - m_{c->v},
 * stopping when H [L < 0] = s; OSD-0 orders columns by (L_v, v), keeps the first
 * GF(2)-independent ones and solves H_S e_S = s on them.  All in FP32. */
typedef struct {
  int32_t max_iter;         /* BP iterations T (>= 1) */
  float alpha;              /* scalar scaling of check messages (plain BP) */
  const float* weights_dev; /* NULL, or FP32 [max_iter][edges] per-edge, per-iteration
                               weights (edges in row-major order of H) replacing alpha */
  int32_t use_osd;          /* 1: OSD-0 on shots where BP did not converge */
  /* launch shape (0 = library default; results never depend on these): */
  int32_t bp_threads;       /* threads of a BP team, the workgroup that decodes one shot
                               at a time (multiple of 64, <= 1024) */
  int32_t bp_per_cu;        /* resident BP teams per compute unit */
  int32_t osd_per_cu;       /* resident OSD workgroups per compute unit */
  int32_t bp_global_state;  /* where a shot's BP state lives.  0: LDS while it fits the 160 KB
                               of a compute unit, otherwise device memory as for 1.  1: device
                               memory, one team (workgroup) per shot.  2: device memory, 64
                               shots per workgroup interleaved by lane (each wave runs one
                               record list of the Tanner graph for all 64 shots; a lane whose
                               shot ends takes the next one).  3: device memory, one team per
                               shot, one pass per iteration (L_v rebuilt per edge from the
                               previous states of v's checks; check states double-buffered).
                               All four give identical results.  Other values: TMCS_EINVAL */
  int32_t osd_order;        /* 0: OSD-0.  1..64: OSD-CS of this order (combination sweep,
                               Roffe et al. 2020; the paper's BP-OSD uses order 7): after the
                               full information set S, every weight-1 flip of the other
                               columns T and every weight-2 flip among T's first osd_order
                               columns; the solution of least soft weight sum L_v over its
                               support wins (FP32, ties to the earlier candidate).  Dense
                               elimination only (<= 2048 detectors, <= 16384 columns) */
  int32_t osd_window;       /* 0: dense OSD-0 when H fits (<= 2048 detectors, <= 16384 columns),
                               windowed otherwise; 1..2048: always windowed, with at most this
                               many detectors in a window.  A window holds the first sorted
                               columns (at most 2047) and the detectors they touch; when the
                               syndrome is spanned inside it the result equals the dense OSD-0
                               exactly, otherwise the shot keeps BP's hard decision and is
                               counted in osd_incomplete (flags bit 3) */
  int32_t decode_chunk;     /* shots per internal decoder pass: 0 = as many as keep the OSD
                               posterior staging (4 * cols bytes per shot) under 8 GiB;
                               otherwise a positive multiple of 64 that caps it.  Results
                               never depend on it (each pass ends on its slowest shots, so
                               fewer passes are faster) */
  int32_t bp_sched;         /* how a BP team's lanes share checks and columns (launch shape;
                               results never depend on it): 0 = library default, 1 =
                               longest-processing-time lists, 2 = strided (lane l of P takes
                               items l, l + P, ...: the lanes of a wave touch consecutive
                               checks and columns, so state in device memory is read in
                               whole cache lines) */
  /* optional per-shot outputs (NULL to skip), each indexed by shot of the call: */
  uint8_t* ehat_dev;        /* [n_shots][cols] final correction (0/1 bytes) */
  float* llr_dev;           /* [n_shots][cols] final BP posterior LLRs */
  int32_t* iters_dev;       /* [n_shots] BP iterations (0 for an all-zero syndrome) */
  uint8_t* flags_dev;       /* [n_shots] bit0 converged, bit1 OSD ran, bit2 OSD not in span,
                               bit3 OSD window exhausted (BP's decision kept) */
} tmcs_decoder_cfg;

/* Decode statistics, accumulated on the device (caller zeroes them). */
#define TMCS_BP_HIST_BINS 65
typedef struct {
  uint64_t shots;        /* shots decoded */
  uint64_t nontrivial;   /* shots with a non-zero syndrome */
  uint64_t converged;    /* shots where BP satisfied the syndrome (all-zero syndromes included) */
  uint64_t osd;          /* shots sent to OSD-0 */
  uint64_t not_in_span;  /* OSD shots whose syndrome was not in H's column space */
  uint64_t bp_iters;     /* sum of BP iterations */
  uint64_t osd_incomplete; /* windowed OSD shots whose syndrome was not spanned inside the window */
  uint64_t osd_prefix_retry; /* OSD shots on DEMs within the dense limits whose first sorted
                                columns (127 for DEMs whose elimination basis fits in LDS,
                                else 1023) did not span the syndrome and that were decoded
                                again with a full sort; the result is the dense OSD-0's
                                either way */
  uint64_t bp_iter_hist[TMCS_BP_HIST_BINS]; /* shots by BP iteration count: bin t < 64 counts
                                shots that ran exactly t iterations (0: all-zero syndrome),
                                bin 64 those that ran 64 or more */
} tmcs_decode_stats;

/* Decode det_dev ([rows][ceil(n/64)], as written by tmcs_sample) and write the
 * predicted observable flips pred_obs_dev ([observables][ceil(n/64)]).
 * stats_dev (device, may be NULL) is incremented.  Work is enqueued on stream;
 * the call does not wait for it.  The DEM handle keeps device scratch that grows
 * with the shots of a pass: about 4 * cols bytes per shot for the posteriors
 * handed to OSD (at most 8 GiB; decode_chunk caps it) plus a few words per shot.
 * Calls on one DEM handle share that scratch, so calls that may overlap in time
 * (different streams) need different handles. */
tmcs_status tmcs_decode(const tmcs_dem* d, const tmcs_decoder_cfg* cfg,
                        const uint64_t* det_dev, uint64_t n_shots, uint64_t* pred_obs_dev,
                        tmcs_decode_stats* stats_dev, void* stream);

/* Whole-operation logical error rate (Methods, "Decoding": a shot fails when
 * any of the k observables is predicted wrongly).  Synchronises the stream.
 * The count is accumulated in a one-word device counter that the library
 * allocates once per device on the first call and reuses; calls are serialised
 * by a host lock held until the result is read.
 * n_errors_host receives the failing-shot count, ler = errors / n_shots and
 * sigma = sqrt(ler (1 - ler) / n_shots) (binomial standard deviation). */
tmcs_status tmcs_logical_error_rate(const uint64_t* pred_obs_dev, const uint64_t* obs_dev,
                                    uint32_t k, uint64_t n_shots, uint64_t* n_errors_host,
                                    double* ler, double* sigma, void* stream);

/* The failing-shot count of tmcs_logical_error_rate, added to *n_errors_dev
 * (device uint64) without waiting, so that counts over many calls are read
 * once.  NULL n_errors_dev: TMCS_EINVAL. */
tmcs_status tmcs_count_errors(const uint64_t* pred_obs_dev, const uint64_t* obs_dev, uint32_t k,
                              uint64_t n_shots, uint64_t* n_errors_dev, void* stream);

/* Weighted (neural) min-sum BP, unrolled for T iterations without early stop,
 * for training per-edge per-iteration weights w[t][e] (FP32 [T][edges]).
 *  tmcs_wbp_workspace_size: bytes of device workspace forward/backward need for
 *  n_shots (per-iteration LLRs and compressed check states; the per-edge
 *  messages are recomputed in the backward pass, not stored).
 *  tmcs_wbp_forward: llr_dev receives FP32 [T][n_shots][cols], L_v after every
 *  iteration; the workspace keeps what the backward pass needs.
 *  tmcs_wbp_backward: given dLoss/dL as FP32 [T][n_shots][cols], accumulates
 *  dLoss/dw into grad_w_dev (FP32 [T][edges], caller zeroes it). */
tmcs_status tmcs_wbp_workspace_size(const tmcs_dem* d, int32_t T, uint64_t n_shots,
                                    size_t* bytes);
tmcs_status tmcs_wbp_forward(const tmcs_dem* d, const float* weights_dev, int32_t T,
                             const uint64_t* det_dev, uint64_t n_shots, float* llr_dev,
                             void* workspace_dev, size_t workspace_bytes, void* stream);
tmcs_status tmcs_wbp_backward(const tmcs_dem* d, const float* weights_dev, int32_t T,
                              const uint64_t* det_dev, uint64_t n_shots,
                              const float* grad_llr_dev, float* grad_w_dev,
                              const void* workspace_dev, size_t workspace_bytes,
                              void* stream);
/* Where the forward/backward kernels keep a shot's working state: in LDS when it
 * fits in the 160 KB of a compute unit (default), else in per-workgroup slabs of
 * device memory that the library allocates.  on = 1 uses the device-memory slabs
 * always (process-wide; results are identical either way). */
tmcs_status tmcs_wbp_global_state(int32_t on);

/* Launch-shape autotuner: decodes the caller's syndromes (det_dev, n_shots
 * shots, as for tmcs_decode) with each candidate launch shape - BP threads and
 * workgroups per compute unit, OSD workgroups per compute unit, BP lane
 * schedule - and writes the fastest into cfg's launch fields (the other fields
 * are kept).  Decoder output never depends on these fields.  The choice is
 * cached per (GPU architecture and CU count, DEM shape, decoder settings) for
 * the life of the process: a later call with the same key returns it without
 * decoding.  Synchronises the stream (when it decodes). */
tmcs_status tmcs_autotune(const tmcs_dem* d, const uint64_t* det_dev, uint64_t n_shots,
                          tmcs_decoder_cfg* cfg, void* stream);

/* Batch plans.  A plan preallocates the whole sample -> decode -> count
 * pipeline of one or more items (circuit, DEM, decoder settings, seed,
 * instance id) for batches of batch_shots shots (a multiple of 4096), and with
 * use_graph = 1 captures one batch of every item into a single HIP graph.
 * The items' decoders run together: one BP launch serves every item whose BP
 * state sits in LDS and one every item whose state sits in device memory (per
 * team size), and one launch runs the windowed OSD-0 of every item that uses
 * it, each pulling jobs from all those items in turn; other OSD variants run
 * per item.  (When an item's batch needs more than one decoder pass, the items
 * decode one after another instead.)
 * Each tmcs_plan_run batch processes the next shot range of every item:
 * shots [k B, (k+1) B) on the k-th batch, with the same bits as tmcs_sample /
 * tmcs_decode on that range.  Counts accumulate on the device;
 * tmcs_plan_result synchronises the stream and reads them for one item.
 * Decoder settings must not request per-shot outputs.  Creation runs one
 * untimed warm-up batch (which allocates all scratch) and resets the counts. */
typedef struct tmcs_plan tmcs_plan;
typedef struct {
  const tmcs_circuit* circuit;
  const tmcs_dem* dem;        /* built from circuit */
  tmcs_decoder_cfg cfg;
  uint64_t seed;
  uint32_t instance;
} tmcs_plan_item;
tmcs_status tmcs_plan_create(const tmcs_plan_item* items, int32_t n_items, uint64_t batch_shots,
                             int32_t use_graph, tmcs_plan** out);
/* tmcs_plan_run: n_batches batches on stream.  While kernel timing is enabled
 * (tmcs_timing_enable) the batches run as eager launches of the same kernels on
 * the same buffers instead of graph replays, so that every launch is timed;
 * the results are the same either way. */
tmcs_status tmcs_plan_run(tmcs_plan* p, uint32_t n_batches, void* stream);
tmcs_status tmcs_plan_result(tmcs_plan* p, int32_t item, uint64_t* shots, uint64_t* errors,
                             tmcs_decode_stats* stats, void* stream);
void tmcs_plan_free(tmcs_plan* p);

/* Kernel timing (a tracing aid).  While enabled, every kernel the library
 * launches is bracketed by a pair of HIP events recorded on the stream it runs
 * on.  tmcs_timing_report synchronises on those events and writes a JSON object
 * {"kernel name": [launches, total milliseconds], ...} (same buffer convention as
 * tmcs_circuit_text); tmcs_timing_reset drops the records. */
tmcs_status tmcs_timing_enable(int on);
tmcs_status tmcs_timing_reset(void);
tmcs_status tmcs_timing_report(char* buf, size_t cap, size_t* len);

/* Thread-local description of the last error ("" if none). */
const char* tmcs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TMCS_H */
