"""GPU parity of the BP + OSD-0 decoder against the oracle.

FP32 decisions (iterations, hard decisions, OSD orderings and corrections,
predicted observables) are compared bit for bit with the oracle run in FP32
in the same operation order; LLRs are also compared with the FP64 oracle at
tolerance 1e-4 max(|L|, 1) on shots both precisions decode within 8 iterations.
"""
import numpy as np
import pytest

from oracle.circuits import build_circuit
from oracle.dem import build_dem
from oracle.frame import pack_bits, sample as oracle_sample, unpack_bits
from oracle.osd import Decoder, logical_errors
from workloads import MEMORY, NLCNOT, TELEPORT, WORKLOADS, bb, pstring, sc, with_decoherence

pytestmark = pytest.mark.gpu

CASES = [
    ("sc3-memory", sc(3, MEMORY, 3, 0, 2e-2), 4096 + 300, 30),
    ("sc3-teleport", sc(3, TELEPORT, 2, 2, 8e-3, 2e-2), 2048 + 17, 30),
    ("sc5-nlcnot", sc(5, NLCNOT, 5, 5, 3e-3, 2e-2), 1024 + 5, 30),
    ("bb18-nlcnot", bb("bb18", NLCNOT, 2, 2, 4e-3, 1e-2), 512 + 3, 30),
    ("bb144-memory", bb("bb144", MEMORY, 4, 0, 2e-3), 96, 20),
    ("sc3-nlcnot-decoherence", with_decoherence(sc(3, NLCNOT, 3, 3, 3e-3, 1e-2), 0.03, False), 2048 + 11, 30),
    ("sc3-pstring4", pstring(sc(3, p=4e-3), 4, rounds=2), 1024 + 7, 30),
    # OSD basis widths of the prefix pass not covered above: 156 detectors (3 words) and 336 (6 words)
    ("sc5-teleport", sc(5, TELEPORT, 3, 3, 3e-3, 1e-2), 1024 + 9, 30),
    ("sc7-nlcnot", sc(7, NLCNOT, 3, 3, 2e-3, 1e-2), 512 + 3, 30),
    # 68 observables (17 blocks of [[18,4,4]]): predictions span two observable words
    ("bb18-pstring16", pstring(bb("bb18", p=4e-3), 16, rounds=1), 512 + 3, 30),
]


def _oracle_det(spec, shots, seed=3):
    """Detector and observable bit planes from the oracle's own sampler (device tensors)."""
    import torch
    d, o = oracle_sample(build_circuit(spec), seed, 0, 0, shots)
    det = torch.from_numpy(pack_bits(d).view(np.int64)).cuda()
    obs = torch.from_numpy(pack_bits(o).view(np.int64)).cuda()
    return det, obs


def _run_lib(tmcs, spec, shots, T, seed=3, alpha=1.0, **kw):
    import torch
    c = tmcs.Circuit(spec)
    dem = tmcs.DEM(c)
    det, obs = _oracle_det(spec, shots, seed)
    N = dem.cols
    k = max(c.num_observables, 1)
    w = (shots + 63) // 64
    pred = torch.zeros((k, w), dtype=torch.int64, device="cuda")
    ehat = torch.zeros((shots, N), dtype=torch.uint8, device="cuda")
    llr = torch.zeros((shots, N), dtype=torch.float32, device="cuda")
    iters = torch.zeros(shots, dtype=torch.int32, device="cuda")
    flags = torch.zeros(shots, dtype=torch.uint8, device="cuda")
    stats = tmcs.new_stats()
    dem.decode(det, shots, pred, max_iter=T, alpha=alpha, ehat=ehat, llr=llr, iters=iters,
               flags=flags, stats=stats, **kw)
    pred2 = torch.zeros_like(pred)
    dem.decode(det, shots, pred2, max_iter=T, alpha=alpha, **kw)          # compacted path
    torch.cuda.synchronize()
    out = dict(det=det.cpu().numpy().view(np.uint64), obs=obs.cpu().numpy().view(np.uint64),
               pred=pred.cpu().numpy().view(np.uint64), pred2=pred2.cpu().numpy().view(np.uint64),
               ehat=ehat.cpu().numpy().astype(bool), llr=llr.cpu().numpy(),
               iters=iters.cpu().numpy(), flags=flags.cpu().numpy(), stats=tmcs.read_stats(stats),
               dem=dem, circuit=c)
    ne, ler, sig = tmcs.logical_error_rate(pred, obs, c.num_observables, shots)
    out["n_err"] = ne
    return out


@pytest.mark.parametrize("name,spec,shots,T", CASES, ids=[c[0] for c in CASES])
def test_decoder_parity(gpu_lib, name, spec, shots, T):
    print(f"[decoder] {name} shots={shots} T={T}", flush=True)
    r = _run_lib(gpu_lib, spec, shots, T)
    od, synd = _check_oracle(r, spec, shots, T)
    check_fp64(r, od, synd, T, name)


LANES_CASES = [c for c in CASES if c[0] in ("sc3-memory", "sc5-nlcnot", "bb18-nlcnot", "bb144-memory",
                                            "sc3-nlcnot-decoherence", "bb18-pstring16")]


@pytest.mark.parametrize("mode", [2, 3], ids=["lanes", "one-pass"])
@pytest.mark.parametrize("name,spec,shots,T", LANES_CASES, ids=[c[0] for c in LANES_CASES])
def test_device_state_kernels_parity(gpu_lib, name, spec, shots, T, mode):
    """The device-memory BP variants against the FP32 oracle: 64 shots per
    workgroup with lane-interleaved state (mode 2), and one team per shot with
    one pass per iteration (mode 3, L_v rebuilt per edge).  sc3-memory has shots
    with s = 0 in the uncompacted (per-shot output) path, bb18-pstring16 two
    observable words, bb144-memory columns of degree 3 and more."""
    print(f"[device-state {mode}] {name} shots={shots} T={T}", flush=True)
    r = _run_lib(gpu_lib, spec, shots, T, bp_global_state=mode)
    _check_oracle(r, spec, shots, T)


def _check_oracle(r, spec, shots, T):
    """Every per-shot output of a decoder run equals the FP32 oracle's."""
    oc = build_circuit(spec)
    od = build_dem(oc)
    synd = unpack_bits(r["det"], shots).T
    obs = unpack_bits(r["obs"], shots).T[:, : oc.num_obs]
    dec32 = Decoder(od.H(), od.priors(), od.L(), max_iter=T, dtype=np.float32)
    o32 = dec32.decode(synd, chunk=64)
    conv = (r["flags"] & 1).astype(bool)
    osd = (r["flags"] & 2).astype(bool)
    assert (r["iters"] == o32["iters"]).all()
    assert (conv == o32["converged"]).all()
    assert (osd == o32["osd"]).all()
    assert (r["llr"] == o32["llr"].astype(np.float32)).all()          # bit-exact FP32
    assert (r["ehat"] == o32["e_hat"]).all()                           # BP and OSD-0 corrections
    assert not (r["flags"] & 4).any()
    pred = unpack_bits(r["pred"], shots).T[:, : oc.num_obs]
    assert (pred == o32["pred_obs"]).all()
    assert (r["pred2"] == r["pred"]).all()
    H = od.H().astype(np.int64)
    assert ((r["ehat"].astype(np.int64) @ H.T) % 2 == synd).all()    # every correction explains s
    n_err = int(logical_errors(o32["pred_obs"], obs).sum())
    assert r["n_err"] == n_err
    st = r["stats"]
    assert st["shots"] == shots and st["osd"] == int(osd.sum())
    assert st["converged"] == int(conv.sum())
    assert st["bp_iters"] == int(r["iters"].sum())
    hist = np.bincount(np.minimum(r["iters"], 64), minlength=65)
    assert list(st["bp_iter_hist"]) == list(hist)
    return od, synd


def fp64_along(f32, priors):
    """FP64 arithmetic along a given FP32 trajectory: every iteration's argmin edges
    and signs are those FP32 took (oracle.wbp forward with unit weights saves them),
    the magnitudes and sums are recomputed in FP64.  Returns L [T, S, n]."""
    from oracle.bp import BIG, prior_llr
    g = f32["graph"]
    lam = prior_llr(priors)
    S = f32["L"].shape[1]
    q = np.broadcast_to(lam[g.ev], (S, g.E)).astype(np.float64).copy()
    out = []
    for sv in f32["saved"]:
        amin = sv["amin"]
        ok = amin >= 0
        mu = np.full((S, g.E), BIG)
        rows = np.nonzero(ok)
        mu[rows] = np.abs(q[rows[0], amin[rows]])
        m = mu * sv["sigma"].astype(np.float64)
        L = lam[None, :].repeat(S, axis=0)
        np.add.at(L, (slice(None), g.ev), m)
        q = L[:, g.ev] - m
        out.append(L)
    return np.stack(out)


FP64_ITERS = 8


def check_fp64(r, od, synd, T, name):
    """FP64 reference LLRs (R21).  L64 is FP64 arithmetic along the FP32 run's
    own argmin and sign decisions.  On every non-trivial shot that stops within
    FP64_ITERS iterations: |L32 - L64| <= 1e-4 max(|L64|, 1) for every column, and
    hard decisions identical except where |L64| < 1e-3 (those columns are flagged:
    counted and printed).  Min-sum on a loopy graph amplifies a rounding
    difference about twofold every one or two iterations (the printed profile
    measures it: on these DEMs the FP32/FP64 difference along one trajectory
    reaches 1e-4 between iteration 7 (BB codes) and 14 (surface codes)), so the
    1e-4 bound is checked on shots that stop within 8 iterations; shots that run
    longer are listed with their fraction and are compared bit for bit with the
    FP32 oracle above.  Pure FP64 (its own decisions and stopping point) is
    reported beside."""
    from oracle.wbp import forward as wbp_forward
    nontriv = np.nonzero(r["iters"] > 0)[0]
    if len(nontriv) == 0:
        return
    H, pri = od.H(), od.priors()
    E = int(H.sum())
    it = r["iters"][nontriv]
    Tmax = int(it.max())
    f32 = wbp_forward(H, pri, synd[nontriv], np.ones((Tmax, E), dtype=np.float32), dtype=np.float32)
    L64 = fp64_along(f32, pri)
    idx = np.arange(len(nontriv))
    # the FP32 forward (no early stop) reproduces the decoder's FP32 LLRs at the stopping iteration
    assert (f32["L"][it - 1, idx] == r["llr"][nontriv]).all()
    prof = []
    for t in range(Tmax):
        running = it > t
        e = np.abs(f32["L"][t][running].astype(np.float64) - L64[t][running]) / \
            np.maximum(np.abs(L64[t][running]), 1.0)
        prof.append(float(e.max()) if e.size else 0.0)
    ok = it <= FP64_ITERS
    ref = L64[it - 1, idx][ok]
    got = r["llr"][nontriv][ok].astype(np.float64)
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    small = np.abs(ref) < 1e-3
    flipped = (got < 0) != (ref < 0)
    longer = nontriv[~ok]
    o64 = Decoder(H, pri, od.L(), max_iter=T, dtype=np.float64, use_osd=False).decode(synd, chunk=64)
    other = nontriv[o64["iters"][nontriv] != r["iters"][nontriv]]
    print(f"[fp64] {name}: {int(ok.sum())} of {len(nontriv)} non-trivial shots checked, max rel err "
          f"{rel.max() if rel.size else 0.0:.2e}; flagged |L64| < 1e-3 columns {int(small.sum())}, of which "
          f"{int((small & flipped).sum())} take the other hard decision; {len(longer)} shots "
          f"({100 * len(longer) / len(nontriv):.1f} %) run more than {FP64_ITERS} iterations: "
          f"{longer[:12].tolist()}{' ...' if len(longer) > 12 else ''}; max rel err by iteration "
          f"{' '.join('%.0e' % x for x in prof)}; pure FP64 stops at another iteration on {len(other)} shots",
          flush=True)
    assert np.all(rel <= 1e-4), float(rel.max())
    assert not (flipped & ~small).any()


def test_decoder_alpha_and_no_osd(gpu_lib):
    spec = sc(5, NLCNOT, 3, 3, 4e-3, 2e-2)
    r = _run_lib(gpu_lib, spec, 700, 25, alpha=0.75)
    od = build_dem(build_circuit(spec))
    synd = unpack_bits(r["det"], 700).T
    o32 = Decoder(od.H(), od.priors(), od.L(), max_iter=25, alpha=0.75, dtype=np.float32).decode(synd)
    assert (r["llr"] == o32["llr"].astype(np.float32)).all()
    assert (r["ehat"] == o32["e_hat"]).all()


def test_decoder_full_size_sampled(gpu_lib):
    """sc5 non-local CNOT at 10^6 shots, bench launch shape: oracle on sampled shots."""
    import torch
    w = WORKLOADS["sc5_nlcnot"]
    spec = w.specs[0]
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    N = w.shots
    det, obs = c.alloc_outputs(N)
    c.sample(w.seed, 0, 0, N, det, obs)
    pred = torch.zeros_like(obs)
    stats = gpu_lib.new_stats()
    dem.decode(det, N, pred, max_iter=w.bp_iters, stats=stats)
    ne, ler, sig = gpu_lib.logical_error_rate(pred, obs, c.num_observables, N)
    torch.cuda.synchronize()
    st = gpu_lib.read_stats(stats)
    print(f"[decoder-full] errors={ne} ler={ler:.3e} stats={st}", flush=True)
    assert st["shots"] == N and st["not_in_span"] == 0
    p = pred.cpu().numpy().view(np.uint64)
    oc = build_circuit(spec)
    od = build_dem(oc)
    dec = Decoder(od.H(), od.priors(), od.L(), max_iter=w.bp_iters, dtype=np.float32)
    rng = np.random.default_rng(0)
    words = np.sort(rng.choice(N // 64, size=12, replace=False))
    for wd in words:
        synd, _ = oracle_sample(oc, w.seed, 0, int(wd) * 64, 64)     # the oracle's own bits of these shots
        o = dec.decode(synd.T)
        got = unpack_bits(p[:, wd:wd + 1], 64).T[:, : od.num_obs]
        assert (got == o["pred_obs"]).all()


@pytest.mark.parametrize("name,spec,shots", [
    ("bb18-nlcnot", bb("bb18", NLCNOT, 2, 2, 4e-3, 1e-2), 700),
    ("sc5-nlcnot", sc(5, NLCNOT, 5, 5, 3e-3, 2e-2), 3000),
], ids=["bb18-nlcnot", "sc5-nlcnot"])
def test_decoder_launch_shape_invariance(gpu_lib, name, spec, shots):
    """Corrections and predictions do not depend on launch shapes or work order."""
    import torch
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    det, obs = c.alloc_outputs(shots)
    c.sample(5, 0, 0, shots, det, obs)
    ref = None
    for kw in (dict(), dict(bp_threads=64, bp_per_cu=2, osd_per_cu=1),
               dict(bp_threads=256, bp_per_cu=16, osd_per_cu=8), dict(bp_threads=1024, osd_per_cu=3),
               dict(bp_global_state=1), dict(bp_global_state=1, bp_threads=128, bp_per_cu=3),
               dict(bp_global_state=2), dict(bp_global_state=2, bp_sched=1, bp_per_cu=2),
               dict(bp_global_state=3), dict(bp_global_state=3, bp_threads=256, bp_per_cu=4)):
        for full in (True, False):
            pred = torch.zeros_like(obs)
            ehat = torch.zeros((shots, dem.cols), dtype=torch.uint8, device="cuda") if full else None
            dem.decode(det, shots, pred, max_iter=30, ehat=ehat, **kw)
            torch.cuda.synchronize()
            p = pred.cpu().numpy()
            if ref is None:
                ref, ref_e = p, ehat.cpu().numpy()
            assert (p == ref).all(), (kw, full)
            if full:
                assert (ehat.cpu().numpy() == ref_e).all(), kw


def test_osd_prefix_retry_matches_oracle(gpu_lib):
    """Dense OSD-0 first eliminates on the 127 smallest keys and re-runs the full
    sort when that prefix does not span s.  At p = 1e-2 some shots need the
    early stop past column 127 of the (L, v) order (counted here from the
    decoder's own FP32 posteriors): they must be retried, and every
    correction must still equal the oracle's BP-OSD."""
    import torch
    from oracle.osd import column_ints
    from test_gpu_osd_window import _early_stop
    spec = sc(5, NLCNOT, 5, 5, 1e-2, 2e-2)
    shots, T = 512, 30
    print(f"[osd-prefix] sc5 p=1e-2 shots={shots}", flush=True)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    det, obs = _oracle_det(spec, shots)
    pred = torch.zeros_like(obs)
    ehat = torch.zeros((shots, dem.cols), dtype=torch.uint8, device="cuda")
    llr = torch.zeros((shots, dem.cols), dtype=torch.float32, device="cuda")
    flags = torch.zeros(shots, dtype=torch.uint8, device="cuda")
    stats = gpu_lib.new_stats()
    dem.decode(det, shots, pred, max_iter=T, ehat=ehat, llr=llr, flags=flags, stats=stats)
    torch.cuda.synchronize()
    oc = build_circuit(spec)
    od = build_dem(oc)
    synd = unpack_bits(det.cpu().numpy().view(np.uint64), shots).T
    o32 = Decoder(od.H(), od.priors(), od.L(), max_iter=T, dtype=np.float32).decode(synd, chunk=64)
    e = ehat.cpu().numpy().astype(bool)
    assert (e == o32["e_hat"]).all()
    assert (unpack_bits(pred.cpu().numpy().view(np.uint64), shots).T[:, : od.L().shape[0]] == o32["pred_obs"]).all()
    st = gpu_lib.read_stats(stats)
    cols = column_ints(od.H())
    L = llr.cpu().numpy()
    late = sum(_early_stop(cols, synd[i], L[i])[0] >= 127 for i in np.nonzero(flags.cpu().numpy() & 2)[0])
    print(f"[osd-prefix] osd {st['osd']} retried {st['osd_prefix_retry']} early stops past 127: {late}", flush=True)
    assert late > 0 and st["osd_prefix_retry"] >= late


@pytest.mark.parametrize("name,spec,shots", [
    ("sc5-nlcnot", sc(5, NLCNOT, 3, 3, 4e-3, 2e-2), 1024 + 3),
    ("bb18-nlcnot", bb("bb18", NLCNOT, 2, 2, 4e-3, 1e-2), 512 + 5),
], ids=["sc5-nlcnot", "bb18-nlcnot"])
def test_osd_cs_matches_oracle(gpu_lib, name, spec, shots):
    """OSD-CS of order 7 (the paper's BP-OSD order) against the oracle's: every
    correction and prediction equal, on oracle-sampled syndromes."""
    import torch
    T = 30
    print(f"[osd-cs] {name} shots={shots}", flush=True)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    det, obs = _oracle_det(spec, shots)
    outs = []
    for order in (7, 0):
        pred = torch.zeros_like(obs)
        ehat = torch.zeros((shots, dem.cols), dtype=torch.uint8, device="cuda")
        flags = torch.zeros(shots, dtype=torch.uint8, device="cuda")
        dem.decode(det, shots, pred, max_iter=T, ehat=ehat, flags=flags, osd_order=order)
        pred2 = torch.zeros_like(obs)
        dem.decode(det, shots, pred2, max_iter=T, osd_order=order)          # compacted path
        torch.cuda.synchronize()
        outs.append((ehat.cpu().numpy().astype(bool), pred.cpu().numpy(), pred2.cpu().numpy(), flags.cpu().numpy()))
    e_cs, p_cs, p2_cs, flags = outs[0]
    assert (p2_cs == p_cs).all()
    oc = build_circuit(spec)
    od = build_dem(oc)
    synd = unpack_bits(det.cpu().numpy().view(np.uint64), shots).T
    o = Decoder(od.H(), od.priors(), od.L(), max_iter=T, dtype=np.float32, osd_order=7).decode(synd, chunk=64)
    assert (e_cs == o["e_hat"]).all()
    assert (unpack_bits(p_cs.view(np.uint64), shots).T[:, : od.L().shape[0]] == o["pred_obs"]).all()
    assert ((e_cs.astype(np.int64) @ od.H().T.astype(np.int64)) % 2 == synd).all()
    osd = (flags & 2).astype(bool)
    changed = (e_cs != outs[1][0]).any(axis=1)
    print(f"[osd-cs] {name}: OSD shots {int(osd.sum())}, corrections changed by CS {int(changed.sum())}", flush=True)
    assert osd.sum() > 10 and changed.sum() > 0 and not (changed & ~osd).any()


def test_several_decoder_passes_equal_one(gpu_lib):
    """Shots split over several internal passes (at most 4096, 1024 or 64 shots
    each; 3 x 4096 + 77 shots, so the last pass is ragged) give the same
    predictions, per-shot outputs and statistics as a single pass, on both the
    full path (per-shot outputs) and the compacted one.  The single pass itself
    is compared with the oracle in test_decoder_parity."""
    import torch
    spec = sc(5, NLCNOT, 5, 5, 3e-3, 2e-2)
    shots, T = 3 * 4096 + 77, 30
    print(f"[decoder] passes sc5-nlcnot shots={shots}", flush=True)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    det, obs = c.alloc_outputs(shots)
    c.sample(5, 0, 0, shots, det, obs)
    N, k, w = dem.cols, max(c.num_observables, 1), (shots + 63) // 64

    def run(chunk):
        pred = torch.zeros((k, w), dtype=torch.int64, device="cuda")
        ehat = torch.zeros((shots, N), dtype=torch.uint8, device="cuda")
        llr = torch.zeros((shots, N), dtype=torch.float32, device="cuda")
        iters = torch.zeros(shots, dtype=torch.int32, device="cuda")
        flags = torch.zeros(shots, dtype=torch.uint8, device="cuda")
        stats = gpu_lib.new_stats()
        dem.decode(det, shots, pred, max_iter=T, ehat=ehat, llr=llr, iters=iters, flags=flags, stats=stats,
                   decode_chunk=chunk)
        pred2 = torch.zeros_like(pred)
        stats2 = gpu_lib.new_stats()
        dem.decode(det, shots, pred2, max_iter=T, stats=stats2, decode_chunk=chunk)     # compacted path
        torch.cuda.synchronize()
        return dict(pred=pred.cpu(), pred2=pred2.cpu(), ehat=ehat.cpu(), llr=llr.cpu(), iters=iters.cpu(),
                    flags=flags.cpu()), gpu_lib.read_stats(stats), gpu_lib.read_stats(stats2)

    ref, st, st2 = run(0)
    assert st["osd"] > 0 and st["shots"] == shots
    assert st2 == st
    assert torch.equal(ref["pred"], ref["pred2"])
    for chunk in (4096, 1024, 64):
        r, s, s2 = run(chunk)
        for key, v in ref.items():
            assert torch.equal(r[key], v), (chunk, key)
        assert s == st and s2 == st, chunk


@pytest.mark.parametrize("T,weighted", [(30, False), (1, False), (2, True), (20, True)],
                         ids=["T30", "T1", "T2-weighted", "T20-weighted"])
def test_lanes_kernel_refills_lanes(gpu_lib, T, weighted):
    """More shots than lanes in flight (256 workgroups x 64 lanes): lanes whose
    shot ends take the next one while the others go on, so lanes of one
    workgroup run different iterations (and, with per-iteration weights,
    different weight rows).  Every per-shot output and the prediction equal the
    team kernel's with its state in LDS, in the per-shot output path and in
    the compacted one; T = 1 and 2 exercise the last-iteration paths.  The
    team kernel with its state in device memory (degree-chunked schedules, no-op
    edges reading per-edge weights of edge 0) is held to the same outputs."""
    import torch
    spec = sc(5, NLCNOT, 5, 5, 3e-3, 2e-2)
    shots = 40000 + 37
    print(f"[lanes-refill] sc5-nlcnot shots={shots} T={T} weighted={weighted}", flush=True)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    det, obs = c.alloc_outputs(shots)
    c.sample(21, 0, 0, shots, det, obs)
    wt = None
    if weighted:
        g = torch.Generator().manual_seed(5)
        wt = (0.5 + 0.6 * torch.rand((T, dem.edges), generator=g)).cuda()

    def run(full, **kw):
        pred = torch.zeros_like(obs)
        st = gpu_lib.new_stats()
        out = dict()
        if full:
            out["llr"] = torch.zeros((shots, dem.cols), dtype=torch.float32, device="cuda")
            out["ehat"] = torch.zeros((shots, dem.cols), dtype=torch.uint8, device="cuda")
            out["iters"] = torch.zeros(shots, dtype=torch.int32, device="cuda")
            out["flags"] = torch.zeros(shots, dtype=torch.uint8, device="cuda")
        dem.decode(det, shots, pred, max_iter=T, weights=wt, stats=st, **out, **kw)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["pred"] = pred.cpu().numpy()
        res["stats"] = gpu_lib.read_stats(st)
        return res

    for full in (True, False):
        ref = run(full)
        for kw in (dict(bp_global_state=2), dict(bp_global_state=2, bp_sched=1, bp_per_cu=2),
                   dict(bp_global_state=3), dict(bp_global_state=1), dict(bp_global_state=1, bp_threads=128)):
            got = run(full, **kw)
            for k in ref:
                if k == "stats":
                    assert got[k] == ref[k], (kw, full)
                else:
                    assert (got[k] == ref[k]).all(), (k, kw, full)
    st = ref["stats"]
    print(f"[lanes-refill] stats {st}", flush=True)
    assert st["nontrivial"] > 16384 and st["osd"] > 0
