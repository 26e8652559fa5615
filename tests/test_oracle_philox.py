"""Pins of the counter-based noise definition (oracle.philox)."""
import os

import numpy as np
import pytest

from oracle.philox import (SB, chain_events, chain_events_scalar, philox4x32_10,
                           philox4x32_10_np, threshold_table)

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((tuple(w[:4]), tuple(w[4:6]), tuple(w[6:10])))
    return rows


def test_philox_known_answers():
    for ctr, key, out in _kat():
        assert philox4x32_10(ctr, key) == out


def test_philox_vectorised_matches_scalar():
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2**32, size=(4, 50), dtype=np.uint64)
    k0, k1 = 0x12345678, 0x9ABCDEF0
    v = philox4x32_10_np(c[0], c[1], c[2], c[3], k0, k1)
    for i in range(50):
        s = philox4x32_10(tuple(int(x) for x in c[:, i]), (k0, k1))
        assert tuple(int(w[i]) for w in v) == s
    for ctr, key, out in _kat():
        v = philox4x32_10_np(*[np.array([x]) for x in ctr], *key)
        assert tuple(int(w[0]) for w in v) == out


def test_threshold_table_is_geometric_tail():
    p = 1e-3
    t = threshold_table(p)
    k = np.arange(1, SB + 1)
    exact = (1 - p) ** k * 2.0**32
    assert np.all(t[1:] >= exact - 1e-3) and np.all(t[1:] <= exact + 1 + 1e-3)
    assert np.all(np.diff(t[1:]) <= 0)
    assert np.all(threshold_table(0.0)[1:] == 2**32)   # p = 0: never an event


@pytest.mark.parametrize("K", [1, 3, 15])
def test_vectorised_chains_match_scalar(K):
    p = 2e-3
    tab = threshold_table(p)
    sites = np.array([0, 7, 123456, 5, 5])
    blocks = np.array([0, 3, 1, 0, 9])
    ch, pos, comp = chain_events(99, 2, sites, blocks, p, K, tab)
    for c in range(sites.size):
        ref = chain_events_scalar(99, 2, int(sites[c]), int(blocks[c]), p, K, tab)
        got = [(int(a), int(b)) for a, b in zip(pos[ch == c], comp[ch == c])]
        assert got == ref


def test_event_statistics():
    """Rate, independence of block positions and uniform components."""
    p = 3e-3
    n_chain = 4000
    ch, pos, comp = chain_events(7, 0, np.arange(n_chain), np.zeros(n_chain, int), p, 15)
    n = ch.size
    expect = n_chain * SB * p
    assert abs(n - expect) < 5 * np.sqrt(expect)
    # positions uniform over the block (chi-square over 16 bins)
    h = np.bincount(pos * 16 // SB, minlength=16)
    chi = ((h - n / 16) ** 2 / (n / 16)).sum()
    assert chi < 45          # 15 dof, p ~ 1e-4
    hc = np.bincount(comp, minlength=15)
    chi = ((hc - n / 15) ** 2 / (n / 15)).sum()
    assert chi < 42          # 14 dof
    # gaps geometric: P(gap >= 1000) = (1-p)^1000
    gaps = np.diff(pos)[np.diff(ch) == 0]
    frac = (gaps > 1000).mean()
    assert abs(frac - (1 - p) ** 1000) < 5 * np.sqrt((1 - p) ** 1000 / gaps.size)
