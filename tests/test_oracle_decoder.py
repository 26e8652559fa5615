"""Pins of the BP / OSD-0 / ML oracle (oracle.bp, oracle.osd, oracle.ml)."""
import itertools

import numpy as np
import pytest

from oracle.bp import decode_bp, prior_llr
from oracle.codes import rank, surface_code
from oracle.ml import expected_ler, ml_ler
from oracle.osd import osd_cs, Decoder, column_ints, logical_errors, osd0


def _tree_H(rng, n_checks):
    """Random tree-shaped factor graph: each new check joins an old variable to 1-2 new ones."""
    edges = []
    nv = 1
    for c in range(n_checks):
        old = int(rng.integers(nv))
        new = list(range(nv, nv + int(rng.integers(1, 3))))
        nv += len(new)
        edges.append([old] + new)
    H = np.zeros((n_checks, nv), dtype=np.uint8)
    for c, vs in enumerate(edges):
        H[c, vs] = 1
    return H


def _min_marginals(H, lam, s):
    n = H.shape[1]
    best = {0: np.full(n, np.inf), 1: np.full(n, np.inf)}
    for bits in itertools.product([0, 1], repeat=n):
        e = np.array(bits)
        if ((H.astype(int) @ e) % 2 != s).any():
            continue
        w = float(lam @ e)
        for v in range(n):
            best[bits[v]][v] = min(best[bits[v]][v], w)
    return best[1] - best[0]


@pytest.mark.parametrize("seed", range(6))
def test_min_sum_exact_on_trees(seed):
    """On a tree, min-sum (alpha = 1) gives exact min-marginals after >= diameter iterations."""
    rng = np.random.default_rng(seed)
    if seed < 3:
        n = 12
        H = np.zeros((n - 1, n), dtype=np.uint8)     # repetition-code chain
        for i in range(n - 1):
            H[i, i] = H[i, i + 1] = 1
    else:
        H = _tree_H(rng, 8)
    n = H.shape[1]
    priors = rng.uniform(0.01, 0.3, size=n)
    lam = prior_llr(priors)
    e = (rng.random(n) < 0.3).astype(int)
    s = (H.astype(int) @ e) % 2
    exact = _min_marginals(H, lam, s)
    r = decode_bp(H, priors, s[None].astype(bool), max_iter=2 * n, early_stop=False)
    assert np.allclose(r["llr"][0], exact, rtol=1e-12, atol=1e-9)


def test_fp32_tracks_fp64():
    c = surface_code(5)
    rng = np.random.default_rng(3)
    priors = rng.uniform(0.01, 0.1, size=c.n)
    e = rng.random((64, c.n)) < 0.08
    s = (e.astype(int) @ c.hz.T.astype(int)) % 2 == 1
    r64 = decode_bp(c.hz, priors, s, 20, alpha=0.75)
    r32 = decode_bp(c.hz, priors, s, 20, alpha=0.75, dtype=np.float32)
    same = r64["iters"] == r32["iters"]
    assert same.mean() > 0.9
    a, b = r64["llr"][same], r32["llr"][same].astype(np.float64)
    assert np.all(np.abs(a - b) <= 1e-4 * np.maximum(1.0, np.abs(a)))


def test_syndrome_zero_is_zero_iterations():
    c = surface_code(3)
    r = decode_bp(c.hz, np.full(c.n, 0.05), np.zeros((2, c.hz.shape[0]), bool), 10)
    assert (r["iters"] == 0).all() and r["converged"].all() and not r["e_hat"].any()


def _gauss_jordan_solve(A, b):
    """Dense textbook solve of A x = b over GF(2) for full-column-rank A."""
    A = A.astype(np.uint8).copy()
    b = b.astype(np.uint8).copy()
    m, k = A.shape
    row = 0
    piv = []
    for col in range(k):
        nz = [r for r in range(row, m) if A[r, col]]
        assert nz
        r = nz[0]
        A[[row, r]] = A[[r, row]]
        b[[row, r]] = b[[r, row]]
        for r2 in range(m):
            if r2 != row and A[r2, col]:
                A[r2] ^= A[row]
                b[r2] ^= b[row]
        piv.append(row)
        row += 1
    assert not b[row:].any()
    return b[:k]


@pytest.mark.parametrize("seed", range(5))
def test_osd0_information_set_and_solution(seed):
    rng = np.random.default_rng(seed)
    m, n = 20, 45
    H = (rng.random((m, n)) < 0.15).astype(np.uint8)
    H[rng.integers(m), :] = 0                     # rank deficient on purpose
    r = rank(H)
    e_true = (rng.random(n) < 0.1)
    s = (H.astype(int) @ e_true) % 2
    llr = rng.normal(size=n)
    llr[:5] = llr[0]                              # ties broken by index
    e, kept, ok = osd0(column_ints(H), r, s, llr)
    assert ok and len(kept) == r
    assert ((H.astype(int) @ e) % 2 == s).all()
    assert set(np.nonzero(e)[0]) <= set(kept)
    # kept = first rank(H) columns that raise the rank, in (llr, index) order
    order = sorted(range(n), key=lambda v: (llr[v], v))
    greedy = []
    for v in order:
        if rank(H[:, greedy + [v]]) > len(greedy):
            greedy.append(v)
        if len(greedy) == r:
            break
    assert kept == greedy
    x = _gauss_jordan_solve(H[:, kept], s)
    assert (e[kept] == x.astype(bool)).all()


def test_osd0_exhaustive_small():
    rng = np.random.default_rng(9)
    H = (rng.random((6, 10)) < 0.4).astype(np.uint8)
    r = rank(H)
    for trial in range(20):
        s = (H.astype(int) @ (rng.random(10) < 0.3)) % 2
        llr = rng.normal(size=10)
        e, kept, ok = osd0(column_ints(H), r, s, llr)
        sols = [x for x in itertools.product([0, 1], repeat=len(kept))
                if ((H[:, kept].astype(int) @ np.array(x)) % 2 == s).all()]
        assert len(sols) == 1 and tuple(e[kept].astype(int)) == sols[0]


@pytest.mark.parametrize("seed,lam", [(0, 3), (1, 7), (2, 7), (3, 40)])
def test_osd_cs_picks_the_lightest_candidate(seed, lam):
    """OSD-CS against its definition, restated with dense algebra: information
    set from GF(2) ranks, every candidate solved by Gauss-Jordan, soft weights in
    FP32 (S in selection order, then the flipped T columns), strict minimum."""
    rng = np.random.default_rng(100 + seed)
    m, n = 14, 30
    H = (rng.random((m, n)) < 0.2).astype(np.uint8)
    H[rng.integers(m), :] = 0
    r = rank(H)
    cols = column_ints(H)
    for trial in range(6):
        s = (H.astype(int) @ (rng.random(n) < 0.15)) % 2
        llr = rng.normal(size=n).astype(np.float32)
        order = sorted(range(n), key=lambda v: (llr[v], v))
        S = []
        for v in order:
            if len(S) < r and rank(H[:, S + [v]]) > len(S):
                S.append(v)
        T = [v for v in order if v not in S]
        cands = [[]] + [[j] for j in T] + [[T[a], T[b]] for a in range(min(lam, len(T)))
                                           for b in range(a + 1, min(lam, len(T)))]
        best = None
        for c in cands:
            rhs = (s + H[:, c].sum(axis=1)) % 2
            x = _gauss_jordan_solve(H[:, S], rhs)
            w = np.float32(0.0)
            for i, v in enumerate(S):
                if x[i]:
                    w = np.float32(w + llr[v])
            for j in c:
                w = np.float32(w + llr[j])
            if best is None or w < best[0]:
                e = np.zeros(n, dtype=bool)
                e[np.array(S)[x.astype(bool)]] = True
                e[c] = True
                best = (w, e)
        e, ok = osd_cs(cols, r, s, llr, lam)
        assert ok and ((H.astype(int) @ e) % 2 == s).all()
        assert (e == best[1]).all(), (seed, trial)
        e0, _, _ = osd0(cols, r, s, llr)
        assert llr[e].sum(dtype=np.float64) <= llr[e0].sum(dtype=np.float64) + 1e-4


def _rep_code_phenomenological(d, rounds):
    """Repetition code with measurement errors: a small space-time DEM."""
    m = (d - 1) * rounds
    cols = []
    for t in range(rounds):
        for q in range(d):               # data flip before round t
            rows = [t * (d - 1) + i for i in (q - 1, q) if 0 <= i < d - 1]
            cols.append((rows, 1 if q == 0 else 0))
        if t < rounds - 1:
            for i in range(d - 1):       # measurement error
                cols.append(([t * (d - 1) + i, (t + 1) * (d - 1) + i], 0))
    H = np.zeros((m, len(cols)), dtype=np.uint8)
    L = np.zeros((1, len(cols)), dtype=np.uint8)
    for j, (rows, o) in enumerate(cols):
        H[rows, j] = 1
        L[0, j] = o
    return H, L


@pytest.mark.parametrize("case", ["sc3_capacity", "rep3x3"])
def test_ler_sampled_vs_exact(case):
    rng = np.random.default_rng(21)
    if case == "sc3_capacity":
        c = surface_code(3)
        H, L = c.hz, c.lz
        priors = np.full(c.n, 0.06)
    else:
        H, L = _rep_code_phenomenological(3, 3)
        priors = rng.uniform(0.03, 0.09, size=H.shape[1])
    dec = Decoder(H, priors, L, max_iter=10)
    lml = ml_ler(H, L, priors)
    lexp = expected_ler(H, L, priors, lambda s: dec.decode(s)["pred_obs"])
    assert lexp >= lml - 1e-12
    N = 40000
    e = rng.random((N, H.shape[1])) < priors
    s = (e.astype(int) @ H.T.astype(int)) % 2 == 1
    o = (e.astype(int) @ L.T.astype(int)) % 2 == 1
    r = dec.decode(s, chunk=4096)
    assert ((r["e_hat"].astype(int) @ H.T.astype(int)) % 2 == s).all()
    err = logical_errors(r["pred_obs"], o).mean()
    sigma = np.sqrt(lexp * (1 - lexp) / N)
    assert abs(err - lexp) < 3 * sigma + 1e-12
