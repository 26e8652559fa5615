"""Graph-captured batch plans and the autotuner against eager calls."""
import numpy as np
import pytest

from workloads import MEMORY, NLCNOT, bb, sc

pytestmark = pytest.mark.gpu


def _eager(tmcs, c, dem, seed, inst, begin, n, T, **kw):
    import torch
    det, obs = c.alloc_outputs(n)
    c.sample(seed, inst, begin, n, det, obs)
    pred = torch.zeros_like(obs)
    st = tmcs.new_stats()
    dem.decode(det, n, pred, max_iter=T, stats=st, **kw)
    ne, _, _ = tmcs.logical_error_rate(pred, obs, c.num_observables, n)
    return ne, tmcs.read_stats(st)


@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "eager-plan"])
def test_plan_matches_eager(gpu_lib, use_graph):
    import torch
    specs = [sc(5, NLCNOT, 3, 3, 3e-3, 2e-2), sc(5, NLCNOT, 3, 3, 6e-3, 2e-2), bb("bb18", MEMORY, 3, 0, 4e-3)]
    B, T = 8192, 30
    circuits = [gpu_lib.Circuit(s) for s in specs]
    dems = [gpu_lib.DEM(c) for c in circuits]
    items = [(c, d, gpu_lib.make_cfg(max_iter=T), 9, i) for i, (c, d) in enumerate(zip(circuits, dems))]
    plan = gpu_lib.Plan(items, B, use_graph=use_graph)
    plan.run(1)
    torch.cuda.synchronize()
    # eager work between replays
    ref = [_eager(gpu_lib, c, d, 9, i, 0, 3 * B, T) for i, (c, d) in enumerate(zip(circuits, dems))]
    plan.run(2)
    for i in range(len(items)):
        r = plan.result(i)
        print(f"[plan] item {i} {r} eager {ref[i]}", flush=True)
        assert r["shots"] == 3 * B
        assert r["errors"] == ref[i][0]
        assert r["stat_shots"] == 3 * B
        assert r["osd"] == ref[i][1]["osd"] and r["converged"] == ref[i][1]["converged"]
        assert r["bp_iters"] == ref[i][1]["bp_iters"]


def test_plan_with_weights_and_windowed_osd_matches_eager(gpu_lib):
    """A captured plan whose items use per-edge, per-iteration BP weights and the
    windowed OSD-0 gives the counts of eager calls with the same configuration."""
    import torch
    specs = [sc(5, NLCNOT, 3, 3, 3e-3, 2e-2), bb("bb18", MEMORY, 3, 0, 4e-3)]
    B, T = 8192, 20
    circuits = [gpu_lib.Circuit(s) for s in specs]
    dems = [gpu_lib.DEM(c) for c in circuits]
    g = torch.Generator().manual_seed(17)
    wts = (0.6 + 0.4 * torch.rand((T, dems[0].edges), generator=g)).cuda()
    kws = [dict(weights=wts), dict(osd_window=16)]
    items = [(c, d, gpu_lib.make_cfg(max_iter=T, **kw), 4, i)
             for i, (c, d, kw) in enumerate(zip(circuits, dems, kws))]
    plan = gpu_lib.Plan(items, B, use_graph=True)
    plan.run(1)
    torch.cuda.synchronize()
    ref = [_eager(gpu_lib, c, d, 4, i, 0, 2 * B, T, **kw)
           for i, (c, d, kw) in enumerate(zip(circuits, dems, kws))]
    plan.run(1)
    for i in range(len(items)):
        r = plan.result(i)
        print(f"[plan-weights] item {i} {r} eager {ref[i]}", flush=True)
        assert r["shots"] == 2 * B and r["errors"] == ref[i][0]
        for k in ("osd", "converged", "bp_iters", "osd_incomplete"):
            assert r[k] == ref[i][1][k], k
    assert ref[0][1]["osd"] > 0 and ref[1][1]["osd"] > 0


def test_autotune_keeps_results(gpu_lib):
    import torch
    spec = sc(5, NLCNOT, 3, 3, 4e-3, 2e-2)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    n = 20000
    det, obs = c.alloc_outputs(n)
    c.sample(1, 0, 0, n, det, obs)
    cfg = gpu_lib.autotune(dem, det, n, gpu_lib.make_cfg(max_iter=30))
    assert cfg.bp_threads in (64, 128, 256, 512, 1024) and cfg.osd_per_cu in (2, 4, 8)
    assert cfg.bp_sched in (1, 2)
    p1 = torch.zeros_like(obs)
    p2 = torch.zeros_like(obs)
    dem.decode(det, n, p1, max_iter=30)
    dem.decode(det, n, p2, max_iter=30, bp_threads=cfg.bp_threads, bp_per_cu=cfg.bp_per_cu,
               osd_per_cu=cfg.osd_per_cu, bp_sched=cfg.bp_sched)
    torch.cuda.synchronize()
    assert (p1.cpu().numpy() == p2.cpu().numpy()).all()
    # the choice is cached per (GPU, DEM shape, settings): a second DEM of the same
    # circuit gets it back at once, without decoding (no syndromes needed)
    import time
    dem2 = gpu_lib.DEM(c)
    t0 = time.perf_counter()
    cfg2 = gpu_lib.autotune(dem2, det, n, gpu_lib.make_cfg(max_iter=30))
    assert time.perf_counter() - t0 < 0.05
    assert (cfg2.bp_threads, cfg2.bp_per_cu, cfg2.osd_per_cu, cfg2.bp_sched) == \
        (cfg.bp_threads, cfg.bp_per_cu, cfg.osd_per_cu, cfg.bp_sched)


@pytest.mark.parametrize("mode", [2, 3], ids=["lanes", "one-pass"])
def test_plan_with_device_state_kernels_matches_eager(gpu_lib, mode):
    """Items whose BP state lives in device memory (mode 2: 64 shots per
    workgroup sharing one slab sized for the largest DEM; mode 3: one pass per
    iteration) share one multi-item launch; the plan's counts equal eager calls
    with the team kernel (state in LDS), with and without per-edge weights."""
    import torch
    specs = [sc(5, NLCNOT, 3, 3, 3e-3, 2e-2), bb("bb18", MEMORY, 3, 0, 4e-3), sc(3, NLCNOT, 3, 3, 5e-3, 2e-2)]
    B, T = 8192, 20
    circuits = [gpu_lib.Circuit(s) for s in specs]
    dems = [gpu_lib.DEM(c) for c in circuits]
    g = torch.Generator().manual_seed(23)
    wts = (0.6 + 0.4 * torch.rand((T, dems[0].edges), generator=g)).cuda()
    kws = [dict(weights=wts), dict(), dict()]
    items = [(c, d, gpu_lib.make_cfg(max_iter=T, bp_global_state=mode, **kw), 6, i)
             for i, (c, d, kw) in enumerate(zip(circuits, dems, kws))]
    plan = gpu_lib.Plan(items, B, use_graph=True)
    plan.run(2)
    torch.cuda.synchronize()
    ref = [_eager(gpu_lib, c, d, 6, i, 0, 3 * B, T, **kw)
           for i, (c, d, kw) in enumerate(zip(circuits, dems, kws))]
    plan.run(1)
    for i in range(len(items)):
        r = plan.result(i)
        print(f"[plan-device-state {mode}] item {i} {r} eager {ref[i]}", flush=True)
        assert r["shots"] == 3 * B and r["errors"] == ref[i][0]
        for k in ("osd", "converged", "bp_iters", "nontrivial", "bp_iter_hist"):
            assert r[k] == ref[i][1][k], k
