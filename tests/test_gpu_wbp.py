"""GPU parity of the weighted-BP training kernels and a training gain test."""
import numpy as np
import pytest

from oracle.circuits import build_circuit
from oracle.dem import build_dem
from oracle.frame import pack_bits, sample as oracle_sample, unpack_bits
from oracle.wbp import backward as oracle_backward
from oracle.wbp import forward as oracle_forward
from workloads import NLCNOT, bb, sc

pytestmark = pytest.mark.gpu


def abs_backward(fwd, G):
    """Per-weight sum of the magnitudes of every term that enters dLoss/dw: the
    oracle's reverse recursion (oracle/wbp.py backward) with each factor replaced
    by its absolute value.  FP32 rounding in the kernel's sums is bounded by a
    small multiple of eps32 times this scale, also where terms cancel."""
    from oracle.bp import BIG
    g = fwd["graph"]
    W = np.abs(np.asarray(fwd["weights"], dtype=np.float64))
    T, S, n = G.shape
    A = np.zeros((T, g.E))
    gq = np.zeros((S, g.E))
    for t in range(T - 1, -1, -1):
        sv = fwd["saved"][t]
        gL = np.abs(np.asarray(G[t], dtype=np.float64))
        np.add.at(gL, (slice(None), g.ev), gq)
        gm = gL[:, g.ev] + gq
        mu = sv["mu"].astype(np.float64)
        finite = mu < BIG / 2
        A[t] = np.sum(np.where(finite, gm * mu, 0.0), axis=0)
        contrib = np.where(finite, gm * W[t][None, :], 0.0)
        gq = np.zeros((S, g.E))
        for s_ in range(S):
            tgt = sv["amin"][s_]
            ok = tgt >= 0
            np.add.at(gq[s_], tgt[ok], contrib[s_, ok])
    return A


def assert_gradient_elementwise(got, ref, scale, label=""):
    """|g - g_ref| <= 1e-4 max(|g_ref|, 0.1 A) for every weight, A = abs_backward's
    scale (so the floor is 1e-5 A: the FP32 sums over shots and checks of a
    weight's terms carry ~K eps32 A error for K summands, K <= a few hundred)."""
    tol = 1e-4 * np.maximum(np.abs(ref), 0.1 * scale)
    bad = np.abs(got - ref) > tol
    worst = float(np.max(np.abs(got - ref) / np.maximum(tol, 1e-300)))
    print(f"[wbp-grad] {label} worst |g - ref| / tol = {worst:.3g} over {ref.size} weights, "
          f"{int((np.abs(ref) < 0.1 * scale).sum())} on the scale floor", flush=True)
    assert not bad.any(), (label, int(bad.sum()), worst)


def _setup(gpu_lib, spec, shots, T, seed=4):
    import torch
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    d, o = oracle_sample(build_circuit(spec), seed, 0, 0, shots)     # inputs from the oracle's sampler
    det = torch.from_numpy(pack_bits(d).view(np.int64)).cuda()
    obs = torch.from_numpy(pack_bits(o).view(np.int64)).cuda()
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.6, 1.4, size=(T, dem.edges)).astype(np.float32)
    wt = torch.from_numpy(w).cuda()
    return c, dem, det, obs, w, wt


@pytest.mark.parametrize("name,spec", [("sc3-nlcnot", sc(3, NLCNOT, 2, 2, 6e-3, 2e-2)),
                                       ("bb18-nlcnot", bb("bb18", NLCNOT, 1, 1, 4e-3, 1e-2))],
                         ids=["sc3-nlcnot", "bb18-nlcnot"])
def test_forward_and_gradient(gpu_lib, name, spec):
    import torch
    T, shots = 6, 128
    c, dem, det, obs, w, wt = _setup(gpu_lib, spec, shots, T)
    ws = torch.empty(dem.wbp_workspace_size(T, shots), dtype=torch.uint8, device="cuda")
    llr = torch.empty((T, shots, dem.cols), dtype=torch.float32, device="cuda")
    dem.wbp_forward(wt, T, det, shots, llr, ws)
    rng = np.random.default_rng(1)
    G = rng.normal(size=(T, shots, dem.cols)).astype(np.float32)
    gw = torch.zeros_like(wt)
    dem.wbp_backward(wt, T, det, shots, torch.from_numpy(G).cuda(), gw, ws)
    torch.cuda.synchronize()
    od = build_dem(build_circuit(spec))
    synd = unpack_bits(det.cpu().numpy().view(np.uint64), shots).T
    f32 = oracle_forward(od.H(), od.priors(), synd, w, dtype=np.float32)
    assert (llr.cpu().numpy() == f32["L"]).all()                    # FP32 forward, bit for bit
    ref = oracle_backward(f32, G.astype(np.float64))                # FP64 arithmetic, same decisions
    got = gw.cpu().numpy().astype(np.float64)
    assert_gradient_elementwise(got, ref, abs_backward(f32, G), name)
    # against the all-FP64 reference gradient: FP64 can take other argmin and sign
    # decisions on near-ties (R19), which moves whole terms, so this is a norm check
    f64 = oracle_forward(od.H(), od.priors(), synd, w.astype(np.float64))
    ref64 = oracle_backward(f64, G.astype(np.float64))
    err64 = np.linalg.norm(got - ref64) / max(np.linalg.norm(ref64), 1e-30)
    assert err64 < 1e-2, err64


def test_unit_weights_match_plain_decoder(gpu_lib):
    """With w = 1 the weighted forward is plain min-sum: same LLRs as the decoder without early stop."""
    import torch
    spec = sc(3, NLCNOT, 2, 2, 6e-3, 2e-2)
    T, shots = 5, 200
    c, dem, det, obs, _, _ = _setup(gpu_lib, spec, shots, T)
    wt = torch.ones((T, dem.edges), dtype=torch.float32, device="cuda")
    ws = torch.empty(dem.wbp_workspace_size(T, shots), dtype=torch.uint8, device="cuda")
    llr = torch.empty((T, shots, dem.cols), dtype=torch.float32, device="cuda")
    dem.wbp_forward(wt, T, det, shots, llr, ws)
    it = torch.zeros(shots, dtype=torch.int32, device="cuda")
    l2 = torch.zeros((shots, dem.cols), dtype=torch.float32, device="cuda")
    pred = torch.zeros_like(obs)
    dem.decode(det, shots, pred, max_iter=T, weights=wt, use_osd=False, llr=l2, iters=it)
    torch.cuda.synchronize()
    iters = it.cpu().numpy()
    L = llr.cpu().numpy()
    for s in range(shots):
        if iters[s] > 0:
            assert (L[iters[s] - 1, s] == l2.cpu().numpy()[s]).all()


def test_training_lowers_the_loss_and_bp_failures(gpu_lib):
    """Weights trained on sampled syndromes beat plain min-sum (alpha = 1) on fresh
    shots, judged by plain BP-OSD: the learned weights send fewer shots to OSD
    (by more than 3 binomial sigma) and do not raise the BP-OSD logical error
    rate by more than 3 sigma."""
    import torch
    from paper_2504_05611_amd import neural_bp
    spec = sc(5, NLCNOT, 3, 3, 5e-3, 2e-2)
    T = 12
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    res = neural_bp.train(c, dem, T, steps=150, batch=512, lr=0.02, seed=21)
    first = float(np.mean(res.losses[:10]))
    last = float(np.mean(res.losses[-10:]))
    print(f"[train] loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < first
    n = 200_000
    plain = neural_bp.evaluate(c, dem, n_shots=n, T=T, use_osd=False, seed=99)
    learned = neural_bp.evaluate(c, dem, n_shots=n, T=T, weights=res.weights, use_osd=False, seed=99)
    print(f"[train] BP-only LER plain {plain['ler']:.4e} learned {learned['ler']:.4e}; "
          f"non-converged plain {1 - plain['converged']:.4e} learned {1 - learned['converged']:.4e}", flush=True)
    assert learned["ler"] < plain["ler"]
    assert learned["converged"] > plain["converged"]
    # the judge: BP-OSD on the same fresh shots
    po = neural_bp.evaluate(c, dem, n_shots=n, T=T, use_osd=True, seed=99)
    lo = neural_bp.evaluate(c, dem, n_shots=n, T=T, weights=res.weights, use_osd=True, seed=99)
    d_osd = po["osd_rate"] - lo["osd_rate"]
    s_osd = np.sqrt((po["osd_rate"] * (1 - po["osd_rate"]) + lo["osd_rate"] * (1 - lo["osd_rate"])) / n)
    s_ler = np.sqrt((po["ler"] * (1 - po["ler"]) + lo["ler"] * (1 - lo["ler"])) / n)
    print(f"[train] BP-OSD LER plain {po['ler']:.4e} learned {lo['ler']:.4e} (sigma {s_ler:.1e}); "
          f"OSD rate plain {po['osd_rate']:.4f} learned {lo['osd_rate']:.4f} (sigma {s_osd:.1e})", flush=True)
    assert d_osd > 3 * s_osd
    assert lo["ler"] <= po["ler"] + 3 * s_ler


def test_state_in_device_memory_matches_lds(gpu_lib):
    """The device-memory variant of the training kernels (used when a shot's state
    exceeds LDS) gives the LDS variant's forward bit for bit and its gradient up
    to the order of FP32 atomic additions."""
    import torch
    spec = bb("bb18", NLCNOT, 1, 1, 4e-3, 1e-2)
    T, shots = 5, 96
    c, dem, det, obs, w, wt = _setup(gpu_lib, spec, shots, T)
    G = torch.from_numpy(np.random.default_rng(3).normal(size=(T, shots, dem.cols)).astype(np.float32)).cuda()
    out = []
    try:
        for gs in (False, True):
            gpu_lib.wbp_global_state(gs)
            ws = torch.empty(dem.wbp_workspace_size(T, shots), dtype=torch.uint8, device="cuda")
            llr = torch.empty((T, shots, dem.cols), dtype=torch.float32, device="cuda")
            dem.wbp_forward(wt, T, det, shots, llr, ws)
            gw = torch.zeros_like(wt)
            dem.wbp_backward(wt, T, det, shots, G, gw, ws)
            torch.cuda.synchronize()
            out.append((llr.cpu().numpy(), gw.cpu().numpy().astype(np.float64)))
    finally:
        gpu_lib.wbp_global_state(False)
    assert (out[0][0] == out[1][0]).all()
    assert np.linalg.norm(out[0][1] - out[1][1]) <= 1e-5 * np.linalg.norm(out[0][1])


def test_training_kernels_at_d15(gpu_lib):
    """d = 15 non-local CNOT of the mixed batch: the per-shot state (~245 KB
    forward, ~370 KB backward) exceeds LDS, so the kernels use device memory;
    forward against the oracle in FP32 bit for bit, gradient against the oracle's.
    The oracle's DEM comes from tests/golden/dem_sc15_nlcnot_p1e-3.npz."""
    import os
    import torch
    from workloads import WORKLOADS
    w_ = WORKLOADS["sc_nlcnot_mixed"]
    inst, spec = next((i, s) for i, s in enumerate(w_.specs) if s.d == 15 and s.p == 1e-3)
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "dem_sc15_nlcnot_p1e-3.npz"))
    m, ncol = int(g["num_dets"]), len(g["priors"])
    H = np.zeros((m, ncol), dtype=np.uint8)
    cp = g["col_ptr"]
    for j in range(ncol):
        H[g["rows"][cp[j]:cp[j + 1]], j] = 1
    T, shots = 3, 4
    print(f"[wbp-d15] m={m} cols={ncol}", flush=True)
    c, dem, det, obs, w, wt = _setup(gpu_lib, spec, shots, T)
    assert dem.rows == m and dem.cols == ncol
    ws = torch.empty(dem.wbp_workspace_size(T, shots), dtype=torch.uint8, device="cuda")
    llr = torch.empty((T, shots, dem.cols), dtype=torch.float32, device="cuda")
    dem.wbp_forward(wt, T, det, shots, llr, ws)
    G = np.random.default_rng(5).normal(size=(T, shots, dem.cols)).astype(np.float32)
    gw = torch.zeros_like(wt)
    dem.wbp_backward(wt, T, det, shots, torch.from_numpy(G).cuda(), gw, ws)
    torch.cuda.synchronize()
    synd = unpack_bits(det.cpu().numpy().view(np.uint64), shots).T
    f32 = oracle_forward(H, g["priors"], synd, w, dtype=np.float32)
    assert (llr.cpu().numpy() == f32["L"]).all()
    ref = oracle_backward(f32, G.astype(np.float64))
    got = gw.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-4 * max(np.linalg.norm(ref), 1e-30)


def test_stored_teleport_weights_lower_the_bposd_ler(gpu_lib):
    """The learned weights shipped for the BB [[144,12,12]] teleportation (T = 20,
    trained on 10^7 syndromes sampled by the library, stored in FP16), judged by
    plain BP-OSD on 2^18 fresh shots: the logical error rate drops by more than 3
    binomial sigma."""
    import os
    import torch
    from paper_2504_05611_amd import neural_bp
    from workloads import WORKLOADS
    w = WORKLOADS["bb144_teleport"]
    spec = w.specs[0]
    path = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_2504_05611_amd", "weights",
                        neural_bp.weights_name(spec, w.bp_iters) + ".npz")
    z = np.load(path)
    assert int(z["train_syndromes"]) >= 10_000_000
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    wt = torch.from_numpy(z["weights"].astype(np.float32)).cuda()
    assert tuple(wt.shape) == (w.bp_iters, dem.edges)
    n = 1 << 18
    plain = neural_bp.evaluate(c, dem, n_shots=n, T=w.bp_iters, use_osd=True, seed=77)
    learned = neural_bp.evaluate(c, dem, n_shots=n, T=w.bp_iters, weights=wt, use_osd=True, seed=77)
    s = np.sqrt((plain["ler"] * (1 - plain["ler"]) + learned["ler"] * (1 - learned["ler"])) / n)
    print(f"[teleport-weights] LER plain {plain['ler']:.4e} learned {learned['ler']:.4e} (sigma {s:.1e}); "
          f"OSD rate plain {plain['osd_rate']:.4f} learned {learned['osd_rate']:.4f}", flush=True)
    assert plain["ler"] - learned["ler"] > 3 * s
