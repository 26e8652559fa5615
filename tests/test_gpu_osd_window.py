"""Windowed OSD-0 against the oracle.

OSD-0 keeps the first GF(2)-independent columns in (L_v, v) order and stops
once the syndrome s lies in their span; the result depends only on the sorted
prefix up to that point.  The windowed kernel works on the first (at most
2047) sorted columns, cut where the detectors they touch would exceed the
window's row limit.  Kept columns vanish outside those detectors, so when s
is spanned inside the window the correction must equal the full OSD-0's bit
for bit; otherwise the shot keeps BP's hard decision and sets flags bit 3.

`_early_stop` below states, independently of the kernel, where the early stop
falls for given posteriors (an XOR basis over Python integers, as in the
oracle's OSD-0): a shot must be complete exactly when the columns up to and
including that point touch at most `osd_window` detectors.  The posteriors
fed to the oracle's OSD-0 are the decoder's own FP32 ones (BP itself is
compared bit for bit with the oracle in test_gpu_decoder.py).
"""
import numpy as np
import pytest

from oracle.circuits import build_circuit
from oracle.codes import rank as gf2_rank
from oracle.dem import build_dem
from oracle.frame import pack_bits, sample as oracle_sample, unpack_bits
from oracle.osd import Decoder, column_ints, osd0
from workloads import NLCNOT, WORKLOADS, sc

pytestmark = pytest.mark.gpu


def _early_stop(cols, synd_bits, llr):
    """(position of the column after which s is spanned, rows touched by columns 0..position)."""
    n = len(cols)
    order = np.lexsort((np.arange(n), np.asarray(llr)))
    s = 0
    for r in np.nonzero(synd_bits)[0]:
        s |= 1 << int(r)
    basis = {}
    touched = 0
    for pos, v in enumerate(order):
        touched |= cols[int(v)]
        x = cols[int(v)]
        while x and (x.bit_length() - 1) in basis:
            x ^= basis[x.bit_length() - 1]
        if not x:
            continue
        basis[x.bit_length() - 1] = x
        y = s
        while y and (y.bit_length() - 1) in basis:
            y ^= basis[y.bit_length() - 1]
        if not y:
            return pos, bin(touched).count("1")
    return n, bin(touched).count("1")


def _decode(tmcs, dem, det, shots, T, **kw):
    import torch
    N = dem.cols
    pred = torch.zeros((max(dem.info["obs"], 1), (shots + 63) // 64), dtype=torch.int64, device="cuda")
    ehat = torch.zeros((shots, N), dtype=torch.uint8, device="cuda")
    llr = torch.zeros((shots, N), dtype=torch.float32, device="cuda")
    flags = torch.zeros(shots, dtype=torch.uint8, device="cuda")
    stats = tmcs.new_stats()
    dem.decode(det, shots, pred, max_iter=T, ehat=ehat, llr=llr, flags=flags, stats=stats, **kw)
    pred2 = torch.zeros_like(pred)
    dem.decode(det, shots, pred2, max_iter=T, **kw)                  # compacted path, no per-shot outputs
    torch.cuda.synchronize()
    return dict(pred=pred.cpu().numpy().view(np.uint64), pred2=pred2.cpu().numpy().view(np.uint64),
                ehat=ehat.cpu().numpy().astype(bool), llr=llr.cpu().numpy(), flags=flags.cpu().numpy(),
                stats=tmcs.read_stats(stats))


def _bp_pred(llr, L):
    return ((llr < 0).astype(np.int64) @ L.T.astype(np.int64)) % 2 == 1


def test_window_covering_h_equals_oracle_osd(gpu_lib):
    """d = 5 non-local CNOT (264 detectors, 1183 columns): a window that holds
    every column reproduces the full BP-OSD of the oracle on every shot."""
    import torch
    spec = sc(5, NLCNOT, 5, 5, 3e-3, 2e-2)
    shots, T = 1024 + 5, 30
    print(f"[osd-window] sc5 full window shots={shots}", flush=True)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    d_or, o_or = oracle_sample(build_circuit(spec), 3, 0, 0, shots)
    det = torch.from_numpy(pack_bits(d_or).view(np.int64)).cuda()
    r = _decode(gpu_lib, dem, det, shots, T, osd_window=2048)
    od = build_dem(build_circuit(spec))
    o32 = Decoder(od.H(), od.priors(), od.L(), max_iter=T, dtype=np.float32).decode(d_or.T, chunk=64)
    osd = (r["flags"] & 2).astype(bool)
    assert osd.sum() > 20
    assert (osd == o32["osd"]).all()
    assert not (r["flags"] & 12).any()
    assert (r["ehat"] == o32["e_hat"]).all()
    assert (unpack_bits(r["pred"], shots).T[:, : od.L().shape[0]] == o32["pred_obs"]).all()
    assert (r["pred2"] == r["pred"]).all()
    assert r["stats"]["osd_incomplete"] == 0


def test_small_window_flags_exactly_the_shots_it_cannot_span(gpu_lib):
    """Same DEM, windows of 12 and 24 detectors: a shot is complete exactly when
    the sorted columns up to the early stop touch at most that many detectors;
    complete shots equal the oracle's OSD-0, the others keep BP's decision."""
    import torch
    spec = sc(5, NLCNOT, 5, 5, 3e-3, 2e-2)
    shots, T = 1024 + 5, 30
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    d_or, _ = oracle_sample(build_circuit(spec), 3, 0, 0, shots)
    det = torch.from_numpy(pack_bits(d_or).view(np.int64)).cuda()
    od = build_dem(build_circuit(spec))
    H, Lm = od.H(), od.L()
    cols = column_ints(H)
    rk = gf2_rank(H)
    seen = {True: 0, False: 0}
    for cap in (12, 24):
        print(f"[osd-window] sc5 window rows={cap}", flush=True)
        r = _decode(gpu_lib, dem, det, shots, T, osd_window=cap)
        inc = (r["flags"] & 8).astype(bool)
        assert r["stats"]["osd_incomplete"] == int(inc.sum())
        assert not (inc & ~(r["flags"] & 2).astype(bool)).any()
        pred = unpack_bits(r["pred"], shots).T[:, : Lm.shape[0]]
        for i in np.nonzero(r["flags"] & 2)[0]:
            pos, rows = _early_stop(cols, d_or[:, i], r["llr"][i])
            complete = rows <= cap and pos < dem.cols
            assert inc[i] == (not complete), (cap, i, pos, rows)
            seen[complete] += 1
            if complete:
                e, _, ok = osd0(cols, rk, d_or[:, i], r["llr"][i])
                assert ok and (r["ehat"][i] == e).all()
            else:
                assert (r["ehat"][i] == (r["llr"][i] < 0)).all()
                assert (pred[i] == _bp_pred(r["llr"][i], Lm)).all()
        assert (r["pred2"] == r["pred"]).all()
    assert seen[True] > 0 and seen[False] > 0


def test_sc11_nlcnot_osd_beyond_dense_limits(gpu_lib):
    """d = 11 non-local CNOT of the mixed batch (2760 detectors, 14,413 columns):
    beyond the dense OSD-0's 2048 detectors, so the decoder windows by itself
    (radix selection of the 2047 smallest keys from 14,413)."""
    import torch
    w = WORKLOADS["sc_nlcnot_mixed"]
    spec = next(s for s in w.specs if s.d == 11 and s.p == 1e-3)
    shots = 64
    print(f"[osd-window] sc11 shots={shots}", flush=True)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    oc = build_circuit(spec)
    d_or, o_or = oracle_sample(oc, w.seed, 1, 0, shots)
    det = torch.from_numpy(pack_bits(d_or).view(np.int64)).cuda()
    r = _decode(gpu_lib, dem, det, shots, w.bp_iters)
    od = build_dem(oc)
    H, Lm = od.H(), od.L()
    assert H.shape == (dem.rows, dem.cols) and dem.rows > 2048
    cols = column_ints(H)
    rk = gf2_rank(H)
    osd = np.nonzero(r["flags"] & 2)[0]
    assert len(osd) >= 4
    assert r["stats"]["osd_incomplete"] == 0
    pred = unpack_bits(r["pred"], shots).T[:, : Lm.shape[0]]
    for i in osd:
        e, _, ok = osd0(cols, rk, d_or[:, i], r["llr"][i])
        assert ok and (r["ehat"][i] == e).all(), i
        assert (pred[i] == ((e.astype(np.int64) @ Lm.T.astype(np.int64)) % 2 == 1)).all()
    assert ((r["ehat"].astype(np.int64) @ H.T.astype(np.int64)) % 2 == d_or.T).all()
    assert (r["pred2"] == r["pred"]).all()


def test_mid_first_window_agrees_with_the_small_one(gpu_lib):
    """d = 29 non-local CNOT of the mixed batch at p = 1e-3 (49,560 detectors,
    about 860 expected detection events): by default a 1024-row first window
    runs before the full 2048-row one; an explicit 2048-row window runs a
    512-row first window instead.  Each window is exact whenever it spans the
    syndrome and numbers its rows in order of first touch, so the smaller
    windows' bases are prefixes of the full one's: every shot's correction,
    flags and predicted observables agree, while far fewer shots reach the
    full window after the larger first one."""
    w = WORKLOADS["sc_nlcnot_mixed"]
    idx, spec = next((i, s) for i, s in enumerate(w.specs) if s.d == 29 and s.p == 1e-3)
    shots = 256
    print(f"[osd-window] sc29 first windows shots={shots}", flush=True)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    det, obs = c.alloc_outputs(shots)
    c.sample(w.seed, idx, 0, shots, det, obs)
    a = _decode(gpu_lib, dem, det, shots, w.bp_iters)
    b = _decode(gpu_lib, dem, det, shots, w.bp_iters, osd_window=2048)
    assert int((a["flags"] & 2).astype(bool).sum()) > shots // 2
    assert (a["flags"] == b["flags"]).all()
    assert (a["ehat"] == b["ehat"]).all()
    assert (a["pred"] == b["pred"]).all()
    assert (a["pred2"] == a["pred"]).all() and (b["pred2"] == b["pred"]).all()
    assert a["stats"]["osd_prefix_retry"] < b["stats"]["osd_prefix_retry"]
