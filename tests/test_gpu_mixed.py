"""Parity at the code sizes of the mixed non-local CNOT batch (d = 21 and 29).

The mixed batch's d = 21 and d = 29 circuits exercise three paths no smaller
case reaches: the frame kernel with one 64-shot word per workgroup and more
than 64 KB of LDS (d = 29: 5044 qubits), BP with its per-shot state in device
memory, and the windowed OSD-0 over tens of thousands of columns.  At d/d
rounds the oracle cannot build these DEMs in reasonable time, so the tests use
the same codes with 3 rounds before and after the CNOT (d = 29: 5880 detectors,
31,335 columns), which reach the same paths.  The oracle's DEMs come from
tests/golden/dem_<name>.npz, written by tests/golden/make_dems.py with oracle/
code only.

Checks: sampled detector and observable bits bit for bit; the library's DEM
equal to the oracle's; FP32 BP posteriors, iteration counts and convergence
bit for bit against the oracle's FP32 BP; OSD corrections equal to the
oracle's OSD-0 on the decoder's own posteriors (the windowed OSD flags the
shots whose syndrome its window does not span: those keep BP's decision).
"""
import os
import sys

import numpy as np
import pytest

from oracle.bp import decode_bp
from oracle.circuits import build_circuit
from oracle.codes import rank as gf2_rank
from oracle.frame import pack_bits, sample as oracle_sample, unpack_bits
from oracle.osd import column_ints, osd0
from workloads import WORKLOADS

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
from make_dems import SPECS, path as dem_path  # noqa: E402

pytestmark = pytest.mark.gpu

# (stored DEM, shots decoded against the oracle): the oracle's FP32 BP takes
# ~3.5 s per shot at d = 29 (20 iterations over 62k edges)
LARGE = [("sc21_nlcnot_r3_p1e-3", 16), ("sc29_nlcnot_r3_p1e-3", 8)]


def stored_dem(name):
    """(H, priors, obs_mask, npz); obs_mask is [cols] uint64, or [cols, words] beyond 64 observables."""
    g = np.load(dem_path(name))
    m, n = int(g["num_dets"]), len(g["priors"])
    H = np.zeros((m, n), dtype=np.uint8)
    cp, rows = g["col_ptr"], g["rows"]
    for j in range(n):
        H[rows[cp[j]:cp[j + 1]], j] = 1
    return H, g["priors"], g["obs_mask"], g


def obs_matrix(obs_mask, k):
    """[k, cols] 0/1 matrix from one- or multi-word observable masks."""
    om = obs_mask[:, None] if obs_mask.ndim == 1 else obs_mask
    return np.stack([(om[:, o // 64] >> np.uint64(o % 64)) & np.uint64(1) for o in range(k)]).astype(np.int64)


@pytest.mark.parametrize("name", [n for n, _ in LARGE])
def test_large_sampler_bits(gpu_lib, name):
    """Two 64-shot words inside the fourth noise block, instance 3."""
    import torch
    spec = SPECS[name]
    print(f"[mixed] sampler {name}", flush=True)
    c = gpu_lib.Circuit(spec)
    begin, n = 3 * 4096 + 5 * 64, 128
    det, obs = c.alloc_outputs(n)
    c.sample(1, 3, begin, n, det, obs)
    torch.cuda.synchronize()
    d_or, o_or = oracle_sample(build_circuit(spec), 1, 3, begin, n)
    assert (det.cpu().numpy().view(np.uint64) == pack_bits(d_or)).all()
    assert (obs.cpu().numpy().view(np.uint64)[: c.num_observables] == pack_bits(o_or)).all()


@pytest.mark.parametrize("name,shots", LARGE, ids=[n for n, _ in LARGE])
def test_large_bp_and_windowed_osd(gpu_lib, name, shots):
    import torch
    spec = SPECS[name]
    T = WORKLOADS["sc_nlcnot_mixed"].bp_iters
    print(f"[mixed] decoder {name} shots={shots} T={T}", flush=True)
    H, priors, obs_mask, _ = stored_dem(name)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    h = dem.export()
    assert (dem.rows, dem.cols) == H.shape
    assert (dem.H() == H).all() and (h.priors == priors).all() and (h.obs_mask == obs_mask).all()
    d_or, _ = oracle_sample(build_circuit(spec), 1, 0, 0, shots)
    det = torch.from_numpy(pack_bits(d_or).view(np.int64)).cuda()
    k = c.num_observables

    def run(use_osd, **kw):
        pred = torch.zeros((k, 1), dtype=torch.int64, device="cuda")
        llr = torch.zeros((shots, dem.cols), dtype=torch.float32, device="cuda")
        ehat = torch.zeros((shots, dem.cols), dtype=torch.uint8, device="cuda")
        iters = torch.zeros(shots, dtype=torch.int32, device="cuda")
        flags = torch.zeros(shots, dtype=torch.uint8, device="cuda")
        dem.decode(det, shots, pred, max_iter=T, use_osd=use_osd, llr=llr, ehat=ehat, iters=iters,
                   flags=flags, **kw)
        torch.cuda.synchronize()
        return dict(pred=pred.cpu().numpy().view(np.uint64), llr=llr.cpu().numpy(), iters=iters.cpu().numpy(),
                    ehat=ehat.cpu().numpy().astype(bool), flags=flags.cpu().numpy())

    bp = run(False, bp_global_state=1)
    # the state placements and lane schedules give the same bits
    for kw in (dict(bp_global_state=0), dict(bp_global_state=1, bp_sched=2),
               dict(bp_global_state=1, bp_threads=512, bp_per_cu=2, bp_sched=1),
               dict(bp_global_state=2), dict(bp_global_state=2, bp_sched=1), dict(bp_global_state=3)):
        other = run(False, **kw)
        assert (other["llr"] == bp["llr"]).all() and (other["iters"] == bp["iters"]).all(), kw
    r = decode_bp(H, priors, d_or.T, T, dtype=np.float32)
    print(f"[mixed] {name} iterations {bp['iters']} oracle {r['iters']}", flush=True)
    assert (bp["iters"] == r["iters"]).all()
    assert ((bp["flags"] & 1).astype(bool) == r["converged"]).all()
    assert (bp["llr"] == r["llr"].astype(np.float32)).all()
    # BP + windowed OSD-0: OSD shots equal the oracle's OSD-0 on the decoder's posteriors
    full = run(True)
    assert (full["llr"] == bp["llr"]).all()
    osd = np.nonzero(full["flags"] & 2)[0]
    assert list(osd) == list(np.nonzero(~r["converged"])[0])
    assert len(osd) >= 2, "no OSD shot to compare"
    cols = column_ints(H)
    rk = gf2_rank(H)
    Lm = obs_matrix(obs_mask, k)
    pred = unpack_bits(full["pred"], shots).T[:, :k]
    incomplete = 0
    for i in osd:
        if full["flags"][i] & 8:                 # window exhausted: BP's decision kept
            incomplete += 1
            assert (full["ehat"][i] == (full["llr"][i] < 0)).all()
            continue
        e, _, ok = osd0(cols, rk, d_or[:, i], full["llr"][i])
        assert ok and (full["ehat"][i] == e).all(), i
        assert (pred[i] == ((e.astype(np.int64) @ Lm.T) % 2 == 1)).all()
    assert incomplete < len(osd)
    synd_ok = (full["ehat"].astype(np.int64) @ H.T.astype(np.int64)) % 2 == d_or.T
    complete = ~((full["flags"] & 8).astype(bool))
    assert synd_ok[complete].all()


def test_mixed_batch_plan_equals_eager_and_oracle(gpu_lib):
    """All eight instances of the mixed batch (d in {11, 15, 21, 29} x p in
    {1e-4, 1e-3}, d/d rounds, T = 20, windowed OSD-0) in one graph-captured
    plan: per-instance error, OSD, convergence and iteration counts equal eager
    sample -> decode calls on the same shots, and 16 shots of the d = 11,
    p = 1e-3 instance equal the oracle's FP32 BP-OSD (stored oracle DEM)."""
    import torch
    w = WORKLOADS["sc_nlcnot_mixed"]
    circuits = [gpu_lib.Circuit(s) for s in w.specs]
    dems = [gpu_lib.DEM(c) for c in circuits]
    B = 4096
    print("[mixed] plan of 8 instances", flush=True)
    plan = gpu_lib.Plan([(c, d, gpu_lib.make_cfg(max_iter=w.bp_iters), w.seed, i)
                         for i, (c, d) in enumerate(zip(circuits, dems))], B, use_graph=True)
    plan.run(1)
    torch.cuda.synchronize()
    eager = {}
    for i, (c, d) in enumerate(zip(circuits, dems)):
        det, obs = c.alloc_outputs(B)
        c.sample(w.seed, i, 0, B, det, obs)
        pred = torch.zeros_like(obs)
        st = gpu_lib.new_stats()
        d.decode(det, B, pred, max_iter=w.bp_iters, stats=st)
        ne, _, _ = gpu_lib.logical_error_rate(pred, obs, c.num_observables, B)
        s = gpu_lib.read_stats(st)
        r = plan.result(i)
        print(f"[mixed] d={w.specs[i].d} p={w.specs[i].p} plan errors {r['errors']} osd {r['osd']} "
              f"converged {r['converged']} iters {r['bp_iters']}; eager errors {ne}", flush=True)
        assert r["shots"] == B and r["errors"] == ne
        for key in ("osd", "converged", "bp_iters", "nontrivial", "osd_incomplete", "bp_iter_hist"):
            assert r[key] == s[key], (i, key)
        eager[i] = (det, pred)
    # oracle on 16 shots of the d = 11, p = 1e-3 instance
    i = next(j for j, s in enumerate(w.specs) if s.d == 11 and s.p == 1e-3)
    H, priors, obs_mask, g = stored_dem("sc11_nlcnot_p1e-3")
    assert (dems[i].H() == H).all()
    det, pred = eager[i]
    shots = 16
    synd = unpack_bits(det.cpu().numpy().view(np.uint64)[:, :1], 64).T[:shots]
    k = circuits[i].num_observables
    Lm = obs_matrix(obs_mask, k).astype(np.uint8)
    from oracle.osd import Decoder
    o = Decoder(H, priors, Lm, max_iter=w.bp_iters, dtype=np.float32).decode(synd, chunk=16)
    got = unpack_bits(pred.cpu().numpy().view(np.uint64)[:, :1], 64).T[:shots, :k]
    assert (got == o["pred_obs"]).all()


def test_bb144_pauli_string_weight5(gpu_lib):
    """Pauli-string compute of weight 5 (pattern 1010) on BB [[144,12,12]] blocks,
    one round first: 6 blocks x 12 logicals = 72 observables, so predictions span
    two mask words.  Library DEM equal to the stored oracle DEM; BP-OSD
    predictions of 48 shots equal the oracle's FP32 BP-OSD."""
    import torch
    from oracle.osd import Decoder
    name = "bb144_pstring5_r1_p1e-3"
    spec = SPECS[name]
    T = 30
    H, priors, obs_mask, _ = stored_dem(name)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    k = c.num_observables
    assert k == 72 and obs_mask.shape == (dem.cols, 2)
    h = dem.export()
    assert (dem.H() == H).all() and (h.priors == priors).all() and (h.obs_mask == obs_mask).all()
    shots = 48
    print(f"[mixed] {name}: {dem.rows} detectors, {dem.cols} columns, {shots} shots", flush=True)
    d_or, o_or = oracle_sample(build_circuit(spec), 1, 0, 0, shots)
    det = torch.from_numpy(pack_bits(d_or).view(np.int64)).cuda()
    pred = torch.zeros((k, 1), dtype=torch.int64, device="cuda")
    flags = torch.zeros(shots, dtype=torch.uint8, device="cuda")
    dem.decode(det, shots, pred, max_iter=T, flags=flags)
    torch.cuda.synchronize()
    o = Decoder(H, priors, obs_matrix(obs_mask, k).astype(np.uint8), max_iter=T, dtype=np.float32).decode(
        d_or.T, chunk=16)
    got = unpack_bits(pred.cpu().numpy().view(np.uint64), shots).T[:, :k]
    fl = flags.cpu().numpy()
    complete = ~((fl & 8).astype(bool))            # windowed OSD: shots spanned inside their window
    assert complete.sum() >= shots - 2
    assert (got[complete] == o["pred_obs"][complete]).all()
