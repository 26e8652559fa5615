"""Parity at the shapes of the other benchmark workloads.

* BB [[144,12,12]] memory, 12 rounds, three noise strengths decoded as three
  instances of one graph-captured plan (the batched launch);
* BB [[144,12,12]] teleportation through 144 ebits (plain BP-OSD and the
  weighted-BP kernels, T = 20);
* the surface-code non-local CNOT of the mixed batch at d = 11 (BP with its
  state in LDS and in device memory; its windowed OSD-0 is checked in
  test_gpu_osd_window.py) and d = 15 (BP state in device memory only).

The oracle checks sampled bits bit for bit and decodes sampled 64-shot words
in FP32 (the decoder's precision) in the same operation order.
"""
import numpy as np
import pytest

from oracle.circuits import build_circuit
from oracle.dem import build_dem
from oracle.frame import pack_bits, sample as oracle_sample, unpack_bits
from oracle.bp import decode_bp
from oracle.osd import Decoder
from oracle.wbp import backward as oracle_backward
from oracle.wbp import forward as oracle_forward
from workloads import WORKLOADS

pytestmark = pytest.mark.gpu


def _check_sampler(tmcs, c, spec, seed, inst, begin, n):
    import torch
    det, obs = c.alloc_outputs(n)
    c.sample(seed, inst, begin, n, det, obs)
    torch.cuda.synchronize()
    d_or, o_or = oracle_sample(build_circuit(spec), seed, inst, begin, n)
    assert (det.cpu().numpy().view(np.uint64) == pack_bits(d_or)).all()
    assert (obs.cpu().numpy().view(np.uint64)[: c.num_observables] == pack_bits(o_or)).all()


def test_bb144_memory_three_instances_in_one_plan(gpu_lib):
    import torch
    w = WORKLOADS["bb144_memory"]
    circuits = [gpu_lib.Circuit(s) for s in w.specs]
    dems = [gpu_lib.DEM(c) for c in circuits]
    B, nb = 8192, 2
    plan = gpu_lib.Plan([(c, d, gpu_lib.make_cfg(max_iter=w.bp_iters), w.seed, i)
                         for i, (c, d) in enumerate(zip(circuits, dems))], B, use_graph=True)
    plan.run(nb)
    torch.cuda.synchronize()
    preds = []
    for i, (c, d) in enumerate(zip(circuits, dems)):
        n = nb * B
        det, obs = c.alloc_outputs(n)
        c.sample(w.seed, i, 0, n, det, obs)
        pred = torch.zeros_like(obs)
        st = gpu_lib.new_stats()
        d.decode(det, n, pred, max_iter=w.bp_iters, stats=st)
        ne, _, _ = gpu_lib.logical_error_rate(pred, obs, c.num_observables, n)
        s = gpu_lib.read_stats(st)
        r = plan.result(i)
        print(f"[bb144-memory] p={w.specs[i].p} plan {r} eager errors {ne} {s}", flush=True)
        assert r["shots"] == n and r["errors"] == ne
        assert r["osd"] == s["osd"] and r["converged"] == s["converged"] and r["bp_iters"] == s["bp_iters"]
        preds.append((det.cpu().numpy().view(np.uint64), pred.cpu().numpy().view(np.uint64)))
    # bits of instance 2 on a stretch that crosses a noise block, and two decoded
    # 64-shot words of every instance (one in each replay's shot range)
    _check_sampler(gpu_lib, circuits[2], w.specs[2], w.seed, 2, 4096 - 64, 128)
    for i in range(3):
        oc = build_circuit(w.specs[i])
        od = build_dem(oc)
        dec = Decoder(od.H(), od.priors(), od.L(), max_iter=w.bp_iters, dtype=np.float32)
        _, p = preds[i]
        for wd in (37 + 11 * i, B // 64 + 5 + 7 * i):
            print(f"[bb144-memory] oracle p={w.specs[i].p} word {wd}", flush=True)
            synd, _ = oracle_sample(oc, w.seed, i, wd * 64, 64)
            o = dec.decode(synd.T)
            assert (unpack_bits(p[:, wd:wd + 1], 64).T[:, : od.num_obs] == o["pred_obs"]).all(), (i, wd)


def test_bb144_teleport_decoder_and_weighted_bp(gpu_lib):
    import torch
    w = WORKLOADS["bb144_teleport"]
    spec = w.specs[0]
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    _check_sampler(gpu_lib, c, spec, w.seed, 0, 2 * 4096 - 64, 128)
    n = 4096
    det, obs = c.alloc_outputs(n)
    c.sample(w.seed, 0, 0, n, det, obs)
    pred = torch.zeros_like(obs)
    dem.decode(det, n, pred, max_iter=w.bp_iters)
    torch.cuda.synchronize()
    p = pred.cpu().numpy().view(np.uint64)
    oc = build_circuit(spec)
    od = build_dem(oc)
    dec = Decoder(od.H(), od.priors(), od.L(), max_iter=w.bp_iters, dtype=np.float32)
    wd = 5
    synd, _ = oracle_sample(oc, w.seed, 0, wd * 64, 64)
    o = dec.decode(synd.T)
    assert (unpack_bits(p[:, wd:wd + 1], 64).T[:, : od.num_obs] == o["pred_obs"]).all()
    # weighted BP at this shape and the workload's T = 20: FP32 forward bit for bit,
    # gradient per weight against the FP64-arithmetic reference
    T, shots = w.bp_iters, 2
    rng = np.random.default_rng(3)
    wts = rng.uniform(0.6, 1.4, size=(T, dem.edges)).astype(np.float32)
    wt = torch.from_numpy(wts).cuda()
    ws = torch.empty(dem.wbp_workspace_size(T, shots), dtype=torch.uint8, device="cuda")
    llr = torch.empty((T, shots, dem.cols), dtype=torch.float32, device="cuda")
    d2, _ = oracle_sample(oc, w.seed, 0, 0, shots)
    det2 = torch.from_numpy(pack_bits(d2).view(np.int64)).cuda()
    dem.wbp_forward(wt, T, det2, shots, llr, ws)
    G = rng.normal(size=(T, shots, dem.cols)).astype(np.float32)
    gw = torch.zeros_like(wt)
    dem.wbp_backward(wt, T, det2, shots, torch.from_numpy(G).cuda(), gw, ws)
    torch.cuda.synchronize()
    synd = d2.T
    f32 = oracle_forward(od.H(), od.priors(), synd, wts, dtype=np.float32)
    assert (llr.cpu().numpy() == f32["L"]).all()
    ref = oracle_backward(f32, G.astype(np.float64))
    got = gw.cpu().numpy().astype(np.float64)
    from test_gpu_wbp import abs_backward, assert_gradient_elementwise
    assert_gradient_elementwise(got, ref, abs_backward(f32, G), "bb144-teleport T=20")


def test_sc11_nlcnot_bp_lds_and_device_state(gpu_lib):
    import torch
    w = WORKLOADS["sc_nlcnot_mixed"]
    spec = next(s for s in w.specs if s.d == 11 and s.p == 1e-3)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    _check_sampler(gpu_lib, c, spec, w.seed, 1, 4096 - 64, 128)
    n = 64
    oc = build_circuit(spec)
    d_or, o_or = oracle_sample(oc, w.seed, 1, 0, n)
    det = torch.from_numpy(pack_bits(d_or).view(np.int64)).cuda()
    pred = torch.zeros((c.num_observables, 1), dtype=torch.int64, device="cuda")
    llr = torch.zeros((n, dem.cols), dtype=torch.float32, device="cuda")
    iters = torch.zeros(n, dtype=torch.int32, device="cuda")
    dem.decode(det, n, pred, max_iter=w.bp_iters, use_osd=False, llr=llr, iters=iters)
    torch.cuda.synchronize()
    od = build_dem(oc)
    synd = d_or.T[:16]
    r = decode_bp(od.H(), od.priors(), synd, w.bp_iters, dtype=np.float32)
    assert (iters.cpu().numpy()[:16] == r["iters"]).all()
    assert (llr.cpu().numpy()[:16] == r["llr"].astype(np.float32)).all()
    # the same shots with the BP state in device memory instead of LDS
    llr_g = torch.zeros_like(llr)
    dem.decode(det, n, pred, max_iter=w.bp_iters, use_osd=False, llr=llr_g, bp_global_state=1)
    torch.cuda.synchronize()
    assert (llr_g.cpu().numpy() == llr.cpu().numpy()).all()


def test_sc15_nlcnot_bp_state_in_device_memory(gpu_lib):
    """d = 15: the per-shot BP state (~336 KB) exceeds LDS and lives in device memory.

    The oracle's DEM of this circuit takes minutes to build, so it is read from
    tests/golden/dem_sc15_nlcnot_p1e-3.npz (written by make_dem_sc15_nlcnot.py
    from oracle/ code only)."""
    import os
    import torch
    w = WORKLOADS["sc_nlcnot_mixed"]
    inst, spec = next((i, s) for i, s in enumerate(w.specs) if s.d == 15 and s.p == 1e-3)
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "dem_sc15_nlcnot_p1e-3.npz"))
    m, ncol = int(g["num_dets"]), len(g["priors"])
    H = np.zeros((m, ncol), dtype=np.uint8)
    cp = g["col_ptr"]
    for j in range(ncol):
        H[g["rows"][cp[j]:cp[j + 1]], j] = 1
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    assert dem.rows == m and dem.cols == ncol
    n = 64
    d_or, _ = oracle_sample(build_circuit(spec), w.seed, inst, 0, n)
    det = torch.from_numpy(pack_bits(d_or).view(np.int64)).cuda()
    pred = torch.zeros((c.num_observables, 1), dtype=torch.int64, device="cuda")
    llr = torch.zeros((n, dem.cols), dtype=torch.float32, device="cuda")
    iters = torch.zeros(n, dtype=torch.int32, device="cuda")
    dem.decode(det, n, pred, max_iter=w.bp_iters, use_osd=False, llr=llr, iters=iters)
    torch.cuda.synchronize()
    r = decode_bp(H, g["priors"], d_or.T[:4], w.bp_iters, dtype=np.float32)
    print(f"[sc15] iters {iters.cpu().numpy()[:4]} oracle {r['iters']}", flush=True)
    assert (iters.cpu().numpy()[:4] == r["iters"]).all()
    assert (llr.cpu().numpy()[:4] == r["llr"].astype(np.float32)).all()
