"""Pins of the code constructions (oracle.codes) against Supplementary Table IV."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle.codes import bb_code, kernel, rank, rref, surface_code

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table4.json")))


def _min_logical_weight(hx, hz, wmax):
    """Brute force: least weight of v in ker(H_X) \\ rowspace(H_Z), searched up to wmax."""
    n = hx.shape[1]
    base = rank(hz)
    hx = hx.astype(np.int64)
    for w in range(1, wmax + 1):
        for supp in itertools.combinations(range(n), w):
            v = np.zeros(n, dtype=np.uint8)
            v[list(supp)] = 1
            if (hx @ v % 2).any():
                continue
            if rank(np.vstack([hz, v])) > base:
                return w
    return None


def test_gf2_helpers():
    a = np.array([[1, 1, 0], [0, 1, 1], [1, 0, 1]], dtype=np.uint8)
    assert rank(a) == 2
    r, piv = rref(a)
    assert piv == [0, 1]
    k = kernel(a)
    assert k.shape == (1, 3) and not ((a.astype(int) @ k.T) % 2).any()


@pytest.mark.parametrize("name", ["bb18", "bb36", "bb54", "bb90", "bb144"])
def test_bb_parameters(name):
    n, k, _ = GOLD["bb"][name]
    c = bb_code(name)
    assert c.n == n and c.k == k
    assert not ((c.hx.astype(int) @ c.hz.T.astype(int)) % 2).any()   # CSS
    assert (c.hx.sum(1) == 6).all() and (c.hz.sum(1) == 6).all()
    assert (c.hx.sum(0) == 3).all() and (c.hz.sum(0) == 3).all()
    # logical Z: commute with X checks, independent of Z checks
    assert not ((c.hx.astype(int) @ c.lz.T.astype(int)) % 2).any()
    assert rank(np.vstack([c.hz, c.lz])) == rank(c.hz) + k


def test_bb_schedule_layers_are_permutations():
    c = bb_code("bb144")
    h = c.n // 2
    for layer in c.z_sched + c.x_sched:
        if not layer:
            continue
        data = [dq for _, dq in layer]
        assert len(set(data)) == h and len(layer) == h
    # the layers reproduce H_X and H_Z
    hx = np.zeros_like(c.hx)
    hz = np.zeros_like(c.hz)
    for layer in c.x_sched:
        for r, dq in layer:
            hx[r, dq] ^= 1
    for layer in c.z_sched:
        for r, dq in layer:
            hz[r, dq] ^= 1
    assert (hx == c.hx).all() and (hz == c.hz).all()


def test_bb18_distance_brute_force():
    c = bb_code("bb18")
    assert _min_logical_weight(c.hx, c.hz, 4) == GOLD["bb"]["bb18"][2]


def _isd_logical(hx, hz, wmax, trials, seed):
    """Lee-Brickell information-set search: in random column orders, the
    reduced row-echelon basis of ker(H_X) and the sums of two of its rows; the
    first of weight <= wmax outside rowspace(H_Z) (a logical Z), or None."""
    rng = np.random.default_rng(seed)
    g = kernel(hx)
    kdim, n = g.shape
    rz = rank(hz)
    for _ in range(trials):
        perm = rng.permutation(n)
        r = rref(g[:, perm])[0].astype(np.int64)
        cand = np.array([r[i] for i in range(kdim)] +
                        [r[i] ^ r[j] for i in range(kdim) for j in range(i + 1, kdim)])
        w = cand.sum(axis=1)
        for idx in np.argsort(w, kind="stable"):
            if w[idx] > wmax:
                break
            z = np.zeros(n, dtype=np.uint8)
            z[perm] = cand[idx].astype(np.uint8)
            if rank(np.vstack([hz, z])) > rz:
                return z
    return None


@pytest.mark.parametrize("name", ["bb90", "bb144"])
def test_bb_distance_upper_bound_matches_table4(name):
    """[[90,8,10]] and [[144,12,12]] are too large for the brute force above.
    An information-set search finds a logical Z of exactly Table IV's distance
    (so d <= the table's value), and none lighter in 40 random column orders
    (evidence for equality, not a proof)."""
    c = bb_code(name)
    d = GOLD["bb"][name][2]
    z = _isd_logical(c.hx, c.hz, d, 20, 1)
    assert z is not None and int(z.sum()) == d
    assert not ((c.hx.astype(int) @ z.astype(int)) % 2).any()          # commutes with every X check
    assert rank(np.vstack([c.hz, z])) == rank(c.hz) + 1                  # not a stabilizer
    assert _isd_logical(c.hx, c.hz, d - 1, 40, 2) is None


@pytest.mark.parametrize("d", [3, 5])
def test_surface_code(d):
    c = surface_code(d)
    assert c.n == d * d and c.k == 1
    assert c.hx.shape[0] == c.hz.shape[0] == (d * d - 1) // 2
    assert not ((c.hx.astype(int) @ c.hz.T.astype(int)) % 2).any()
    assert c.n - rank(c.hx) - rank(c.hz) == 1
    assert not ((c.hx.astype(int) @ c.lz.T.astype(int)) % 2).any()
    assert c.lz.sum() == d
    assert _min_logical_weight(c.hx, c.hz, d) == d
    # schedule: every layer touches each qubit at most once
    for t in range(4):
        qs = [("d", dq) for _, dq in c.x_sched[t] + c.z_sched[t]]
        assert len(qs) == len(set(qs))
    # each CX layer reproduces the checks
    hx = np.zeros_like(c.hx)
    for layer in c.x_sched:
        for r, dq in layer:
            hx[r, dq] ^= 1
    assert (hx == c.hx).all()
