"""ctypes binding of libtmcs.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module only converts
Python values and torch device tensors into the C ABI declared in
include/tmcs.h.  Importing it fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtmcs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libtmcs.so is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_2504_05611_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

TMCS_SC, TMCS_BB = 0, 1
TMCS_MEMORY, TMCS_NONLOCAL_CNOT, TMCS_TELEPORT, TMCS_PAULI_STRING = 0, 1, 2, 3
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EUNSUPPORTED",
          5: "ENONDETERMINISTIC"}
INFO_KEYS = ["qubits", "gates_1q", "gates_2q", "meas", "meas_final", "detectors",
             "observables", "noise_sites", "instructions", "code_n", "code_k", "events_per_mshot"]
DEM_KEYS = ["rows", "cols", "obs", "edges", "rank", "undetectable", "max_row_deg", "max_col_deg"]


class TmcsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tmcs {STATUS.get(status, status)}: {msg}")
        self.status = status


class _Spec(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("d", ctypes.c_int32),
                ("bb_l", ctypes.c_int32), ("bb_m", ctypes.c_int32),
                ("bb_a", (ctypes.c_int32 * 2) * 3), ("bb_b", (ctypes.c_int32 * 2) * 3),
                ("op", ctypes.c_int32), ("rounds_before", ctypes.c_int32),
                ("rounds_after", ctypes.c_int32), ("p", ctypes.c_double), ("p_ebit", ctypes.c_double),
                ("ebit_per_step", ctypes.c_int32), ("ebit_rate", ctypes.c_double),
                ("weight", ctypes.c_int32)]


class DecoderCfg(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("weights_dev", ctypes.c_void_p), ("use_osd", ctypes.c_int32),
                ("bp_threads", ctypes.c_int32), ("bp_per_cu", ctypes.c_int32),
                ("osd_per_cu", ctypes.c_int32), ("bp_global_state", ctypes.c_int32),
                ("osd_order", ctypes.c_int32), ("osd_window", ctypes.c_int32),
                ("decode_chunk", ctypes.c_int32), ("bp_sched", ctypes.c_int32),
                ("ehat_dev", ctypes.c_void_p),
                ("llr_dev", ctypes.c_void_p), ("iters_dev", ctypes.c_void_p),
                ("flags_dev", ctypes.c_void_p)]


class DecodeStats(ctypes.Structure):
    _fields_ = [("shots", ctypes.c_uint64), ("nontrivial", ctypes.c_uint64),
                ("converged", ctypes.c_uint64), ("osd", ctypes.c_uint64),
                ("not_in_span", ctypes.c_uint64), ("bp_iters", ctypes.c_uint64),
                ("osd_incomplete", ctypes.c_uint64), ("osd_prefix_retry", ctypes.c_uint64),
                ("bp_iter_hist", ctypes.c_uint64 * 65)]


STATS_WORDS = 8 + 65          # tmcs_decode_stats: 8 counters and the 65-bin BP iteration histogram


class PlanItem(ctypes.Structure):
    _fields_ = [("circuit", ctypes.c_void_p), ("dem", ctypes.c_void_p), ("cfg", DecoderCfg),
                ("seed", ctypes.c_uint64), ("instance", ctypes.c_uint32)]


_vp, _u64, _u32, _i32, _sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_size_t
_SIGS = {
    "tmcs_build_circuit": [ctypes.POINTER(_Spec), ctypes.POINTER(_vp)],
    "tmcs_free_circuit": [_vp],
    "tmcs_circuit_info": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "tmcs_circuit_text": [_vp, ctypes.c_char_p, _sz, ctypes.POINTER(_sz)],
    "tmcs_build_dem": [_vp, ctypes.POINTER(_vp)],
    "tmcs_free_dem": [_vp],
    "tmcs_dem_info": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "tmcs_dem_export": [_vp, _vp, _vp, _vp, _vp],
    "tmcs_dem_distance": [_vp, _i32, _i32, ctypes.c_int64, ctypes.POINTER(_i32)],
    "tmcs_dem_distance_device": [_vp, _i32, _i32, ctypes.c_int64, ctypes.POINTER(_i32), _vp],
    "tmcs_sample": [_vp, _u64, _u32, _u64, _u64, _vp, _vp, _vp],
    "tmcs_sample_async": [_vp, _u64, _u32, _u64, _u64, _vp, _vp, _vp, _vp],
    "tmcs_sample_noalloc": [_vp, _u64, _u32, _u64, _u64, _vp, _vp, _vp, _vp],
    "tmcs_count_errors": [_vp, _vp, _u32, _u64, _vp, _vp],
    "tmcs_decode": [_vp, ctypes.POINTER(DecoderCfg), _vp, _u64, _vp, _vp, _vp],
    "tmcs_logical_error_rate": [_vp, _vp, _u32, _u64, ctypes.POINTER(_u64),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _vp],
    "tmcs_wbp_workspace_size": [_vp, _i32, _u64, ctypes.POINTER(_sz)],
    "tmcs_wbp_forward": [_vp, _vp, _i32, _vp, _u64, _vp, _vp, _sz, _vp],
    "tmcs_wbp_backward": [_vp, _vp, _i32, _vp, _u64, _vp, _vp, _vp, _sz, _vp],
    "tmcs_wbp_global_state": [_i32],
    "tmcs_autotune": [_vp, _vp, _u64, ctypes.POINTER(DecoderCfg), _vp],
    "tmcs_plan_create": [ctypes.POINTER(PlanItem), _i32, _u64, _i32, ctypes.POINTER(_vp)],
    "tmcs_plan_run": [_vp, _u32, _vp],
    "tmcs_plan_result": [_vp, _i32, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(DecodeStats), _vp],
    "tmcs_plan_free": [_vp],
    "tmcs_timing_enable": [ctypes.c_int],
    "tmcs_timing_reset": [],
    "tmcs_timing_report": [_vp, ctypes.c_char_p, _sz, ctypes.POINTER(_sz)][1:],
    "tmcs_last_error": [],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.tmcs_last_error.restype = ctypes.c_char_p
_lib.tmcs_free_circuit.restype = None
_lib.tmcs_free_dem.restype = None
_lib.tmcs_plan_free.restype = None

EXPORTED = sorted(_SIGS)


def _check(st):
    if st != 0:
        raise TmcsError(st, _lib.tmcs_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


def spec_struct(spec) -> _Spec:
    """workloads.CircuitSpec -> C struct."""
    s = _Spec()
    s.code = TMCS_SC if spec.code == "sc" else TMCS_BB
    s.d = spec.d
    if spec.code == "bb":
        from workloads import BB_CODES
        l, m, a, b = BB_CODES[spec.bb]
        s.bb_l, s.bb_m = l, m
        for k in range(3):
            s.bb_a[k][0], s.bb_a[k][1] = a[k]
            s.bb_b[k][0], s.bb_b[k][1] = b[k]
    s.op = {"memory": TMCS_MEMORY, "nlcnot": TMCS_NONLOCAL_CNOT, "teleport": TMCS_TELEPORT,
            "pstring": TMCS_PAULI_STRING}[spec.op]
    s.rounds_before = spec.rounds_before
    s.rounds_after = spec.rounds_after
    s.p = spec.p
    s.p_ebit = spec.p_ebit
    s.ebit_per_step = getattr(spec, "ebit_per_step", 0)
    s.ebit_rate = getattr(spec, "ebit_rate", 0.0)
    s.weight = getattr(spec, "weight", 0)
    return s


class Circuit:
    def __init__(self, spec):
        self.spec = spec
        h = ctypes.c_void_p()
        _check(_lib.tmcs_build_circuit(ctypes.byref(spec_struct(spec)), ctypes.byref(h)))
        self._h = h
        arr = (ctypes.c_int64 * 16)()
        _check(_lib.tmcs_circuit_info(self._h, arr))
        self.info = {k: int(arr[i]) for i, k in enumerate(INFO_KEYS)}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.tmcs_free_circuit(h)
            self._h = None

    @property
    def num_detectors(self):
        return self.info["detectors"]

    @property
    def num_observables(self):
        return self.info["observables"]

    def text(self) -> str:
        n = ctypes.c_size_t()
        _check(_lib.tmcs_circuit_text(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(_lib.tmcs_circuit_text(self._h, buf, n.value + 1, ctypes.byref(n)))
        return buf.value.decode()

    def sample(self, seed, instance, shot_begin, n_shots, det, obs, stream=None):
        """det/obs: int64 device tensors [rows][ceil(n/64)] (bit-packed uint64)."""
        _check(_lib.tmcs_sample(self._h, seed, instance, shot_begin, n_shots, _ptr(det), _ptr(obs),
                                _stream(stream)))

    def sample_async(self, seed, instance, shot_begin, n_shots, det, obs, overflow, stream=None):
        """sample() without waiting; an event-buffer overflow sets the device flag
        `overflow` (int32 tensor of one element, zeroed by the caller)."""
        _check(_lib.tmcs_sample_async(self._h, seed, instance, shot_begin, n_shots, _ptr(det), _ptr(obs),
                                      _ptr(overflow), _stream(stream)))

    def sample_noalloc(self, seed, instance, shot_begin, n_shots, det, obs, overflow, stream=None):
        """sample_async() on the library's fixed device scratch (no allocation); the
        program must already be on the device (an earlier sample/sample_async call)."""
        _check(_lib.tmcs_sample_noalloc(self._h, seed, instance, shot_begin, n_shots, _ptr(det), _ptr(obs),
                                        _ptr(overflow), _stream(stream)))

    def alloc_outputs(self, n_shots, device="cuda"):
        import torch
        w = (n_shots + 63) // 64
        det = torch.empty((self.num_detectors, w), dtype=torch.int64, device=device)
        obs = torch.empty((max(self.num_observables, 1), w), dtype=torch.int64, device=device)
        return det, obs


@dataclass
class DemHost:
    col_ptr: np.ndarray
    row_idx: np.ndarray
    priors: np.ndarray
    obs_mask: np.ndarray


class DEM:
    def __init__(self, circuit: Circuit):
        h = ctypes.c_void_p()
        _check(_lib.tmcs_build_dem(circuit._h, ctypes.byref(h)))
        self._h = h
        self.circuit = circuit
        arr = (ctypes.c_int64 * 16)()
        _check(_lib.tmcs_dem_info(self._h, arr))
        self.info = {k: int(arr[i]) for i, k in enumerate(DEM_KEYS)}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.tmcs_free_dem(h)
            self._h = None

    @property
    def rows(self):
        return self.info["rows"]

    @property
    def cols(self):
        return self.info["cols"]

    @property
    def edges(self):
        return self.info["edges"]

    def distance(self, max_active=8, max_weight=16, max_states=20_000_000, device=False, stream=None) -> int:
        """Fewest mechanisms found forming an undetectable logical error (0: none
        within the limits); exact when max_active >= rows and the budget suffices.
        device=True runs the level-synchronous search on the GPU (max_active <= 16)."""
        w = ctypes.c_int32()
        if device:
            _check(_lib.tmcs_dem_distance_device(self._h, max_active, max_weight, max_states, ctypes.byref(w),
                                                 _stream(stream)))
        else:
            _check(_lib.tmcs_dem_distance(self._h, max_active, max_weight, max_states, ctypes.byref(w)))
        return w.value

    @property
    def obs_words(self):
        return max(1, (self.info["obs"] + 63) // 64)

    def export(self) -> DemHost:
        """Host copy; obs_mask is uint64 [cols] with at most 64 observables, else [cols, words]."""
        n, e = self.info["cols"], self.info["edges"]
        ow = self.obs_words
        cp = np.zeros(n + 1, dtype=np.int32)
        ri = np.zeros(max(e, 1), dtype=np.int32)
        pr = np.zeros(max(n, 1), dtype=np.float64)
        om = np.zeros((max(n, 1), ow), dtype=np.uint64)
        _check(_lib.tmcs_dem_export(self._h, cp.ctypes.data, ri.ctypes.data, pr.ctypes.data, om.ctypes.data))
        return DemHost(cp, ri[:e], pr[:n], om[:n, 0] if ow == 1 else om[:n])

    def L(self) -> np.ndarray:
        """[observables, cols] 0/1 matrix of the columns that flip each observable."""
        om = self.export().obs_mask
        om = om[:, None] if om.ndim == 1 else om
        k = self.info["obs"]
        L = np.zeros((k, self.cols), dtype=np.uint8)
        for o in range(k):
            L[o] = ((om[:, o // 64] >> np.uint64(o % 64)) & np.uint64(1)).astype(np.uint8)
        return L

    def H(self) -> np.ndarray:
        h = self.export()
        H = np.zeros((self.rows, self.cols), dtype=np.uint8)
        for j in range(self.cols):
            H[h.row_idx[h.col_ptr[j]:h.col_ptr[j + 1]], j] = 1
        return H

    def decode(self, det, n_shots, pred, *, max_iter=30, alpha=1.0, weights=None, use_osd=True,
               bp_threads=0, bp_per_cu=0, osd_per_cu=0, bp_global_state=0, osd_order=0, osd_window=0,
               decode_chunk=0, bp_sched=0, ehat=None, llr=None, iters=None, flags=None, stats=None,
               stream=None):
        cfg = DecoderCfg(max_iter, alpha, _ptr(weights), 1 if use_osd else 0, bp_threads,
                         bp_per_cu, osd_per_cu, bp_global_state, osd_order, osd_window, decode_chunk, bp_sched,
                         _ptr(ehat), _ptr(llr), _ptr(iters), _ptr(flags))
        _check(_lib.tmcs_decode(self._h, ctypes.byref(cfg), _ptr(det), n_shots, _ptr(pred), _ptr(stats),
                                _stream(stream)))

    def wbp_workspace_size(self, T, n_shots):
        n = ctypes.c_size_t()
        _check(_lib.tmcs_wbp_workspace_size(self._h, T, n_shots, ctypes.byref(n)))
        return n.value

    def wbp_forward(self, weights, T, det, n_shots, llr, workspace, stream=None):
        _check(_lib.tmcs_wbp_forward(self._h, _ptr(weights), T, _ptr(det), n_shots, _ptr(llr),
                                     _ptr(workspace), workspace.numel() * workspace.element_size(),
                                     _stream(stream)))

    def wbp_backward(self, weights, T, det, n_shots, grad_llr, grad_w, workspace, stream=None):
        _check(_lib.tmcs_wbp_backward(self._h, _ptr(weights), T, _ptr(det), n_shots, _ptr(grad_llr),
                                      _ptr(grad_w), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _stream(stream)))


def wbp_global_state(on=True):
    """Keep the training kernels' per-shot state in device memory (1) or in LDS when it fits (0)."""
    _check(_lib.tmcs_wbp_global_state(1 if on else 0))


def make_cfg(max_iter=30, alpha=1.0, weights=None, use_osd=True, bp_threads=0, bp_per_cu=0,
             osd_per_cu=0, bp_global_state=0, osd_order=0, osd_window=0, decode_chunk=0, bp_sched=0):
    return DecoderCfg(max_iter, alpha, _ptr(weights), 1 if use_osd else 0, bp_threads, bp_per_cu,
                      osd_per_cu, bp_global_state, osd_order, osd_window, decode_chunk, bp_sched,
                      None, None, None, None)


def autotune(dem, det, n_shots, cfg=None, stream=None) -> DecoderCfg:
    """Fastest decoder launch shape for these syndromes (fields of DecoderCfg)."""
    cfg = cfg or make_cfg()
    _check(_lib.tmcs_autotune(dem._h, _ptr(det), n_shots, ctypes.byref(cfg), _stream(stream)))
    return cfg


class Plan:
    """Preallocated (optionally graph-captured) sample -> decode -> count batches.

    items: list of (circuit, dem, DecoderCfg, seed, instance)."""

    def __init__(self, items, batch_shots, use_graph=True):
        self._keep = items
        arr = (PlanItem * len(items))()
        for i, (c, d, cfg, seed, inst) in enumerate(items):
            arr[i].circuit = c._h
            arr[i].dem = d._h
            arr[i].cfg = cfg
            arr[i].seed = seed
            arr[i].instance = inst
        h = ctypes.c_void_p()
        _check(_lib.tmcs_plan_create(arr, len(items), batch_shots, 1 if use_graph else 0, ctypes.byref(h)))
        self._h = h
        self.batch = batch_shots

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.tmcs_plan_free(h)
            self._h = None

    def run(self, n_batches, stream=None):
        _check(_lib.tmcs_plan_run(self._h, n_batches, _stream(stream)))

    def result(self, item=0, stream=None):
        shots = ctypes.c_uint64()
        errs = ctypes.c_uint64()
        st = DecodeStats()
        _check(_lib.tmcs_plan_result(self._h, item, ctypes.byref(shots), ctypes.byref(errs), ctypes.byref(st),
                                     _stream(stream)))
        return dict(shots=shots.value, errors=errs.value, nontrivial=st.nontrivial, converged=st.converged,
                    osd=st.osd, not_in_span=st.not_in_span, bp_iters=st.bp_iters,
                    osd_incomplete=st.osd_incomplete, osd_prefix_retry=st.osd_prefix_retry,
                    stat_shots=st.shots, bp_iter_hist=[int(x) for x in st.bp_iter_hist])


def count_errors(pred, obs, k, n_shots, counter, stream=None):
    """Add the failing-shot count to the device counter (int64 tensor of one element) without waiting."""
    _check(_lib.tmcs_count_errors(_ptr(pred), _ptr(obs), k, n_shots, _ptr(counter), _stream(stream)))


def logical_error_rate(pred, obs, k, n_shots, stream=None):
    ne = ctypes.c_uint64()
    ler = ctypes.c_double()
    sig = ctypes.c_double()
    _check(_lib.tmcs_logical_error_rate(_ptr(pred), _ptr(obs), k, n_shots, ctypes.byref(ne),
                                        ctypes.byref(ler), ctypes.byref(sig), _stream(stream)))
    return ne.value, ler.value, sig.value


def timing_enable(on=True):
    _check(_lib.tmcs_timing_enable(1 if on else 0))


def timing_reset():
    _check(_lib.tmcs_timing_reset())


def timing_report() -> dict:
    """{kernel: (launches, total ms)} for the launches recorded while timing was on."""
    import json
    n = ctypes.c_size_t()
    _check(_lib.tmcs_timing_report(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(_lib.tmcs_timing_report(buf, n.value + 1, ctypes.byref(n)))
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}


def new_stats(device="cuda"):
    import torch
    return torch.zeros(STATS_WORDS, dtype=torch.int64, device=device)


def read_stats(t) -> dict:
    v = t.cpu().numpy().astype(np.uint64)
    return dict(shots=int(v[0]), nontrivial=int(v[1]), converged=int(v[2]), osd=int(v[3]),
                not_in_span=int(v[4]), bp_iters=int(v[5]), osd_incomplete=int(v[6]),
                osd_prefix_retry=int(v[7]), bp_iter_hist=[int(x) for x in v[8:8 + 65]])
