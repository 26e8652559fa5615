"""Counter-based noise: Philox4x32-10 and the block-geometric event definition.

Philox4x32-10 is restated from its published definition (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
32x32->64 multiplies with fixed multipliers, a word permutation, and a Weyl
key schedule bumped between rounds.

The paper samples circuit noise with a stabilizer simulator and does not fix
its random bits (Methods, Simulation).  The reading used here makes every
sampled bit a pure function of (seed, instance, noise site, shot block):

* key = (seed low 32 bits, seed high 32 bits);
  counter = (block b, site s, instance i, call j).  The four words of call j
  are draws 4j .. 4j+3 of the (b, s, i) stream, consumed in order.
* A block is SB = 4096 consecutive shots.
* For event probability p, t_0 = 1, t_k = t_{k-1} * (1 - p) (FP64), and
  T[k] = ceil(t_k * 2**32) for k = 1..SB.  P(u < T[k]) = (1-p)**k, so the
  count g = #{k : u < T[k]} is geometric: the number of event-free shots
  before the next event.
* Per (b, s, i): pos = -1; repeat: draw u, pos += g(u) + 1, stop if
  pos >= SB, else an event at shot b*SB + pos; if the channel has K > 1
  components, draw v and take component (v * K) >> 32.

Parity: pinned by published Philox known-answer vectors and by the
statistics of the generated events (tests/test_oracle_philox.py).
"""
from __future__ import annotations

import math

import numpy as np

SB = 4096  # shots per noise block (part of the bit definition)

_M0 = 0xD2511F53
_M1 = 0xCD9E8D57
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Scalar Philox4x32-10: ctr = 4 uint32, key = 2 uint32 -> 4 uint32."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in ctr)
    k0, k1 = (int(x) & _MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0, c1, c2, c3)


def philox4x32_10_np(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over uint32 arrays (same definition)."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(k0) & _MASK)
    k1 = np.uint64(int(k1) & _MASK)
    m = np.uint64(_MASK)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + _W0) & _MASK)
            k1 = np.uint64((int(k1) + _W1) & _MASK)
        p0 = np.uint64(_M0) * c0
        p1 = np.uint64(_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def threshold_table(p: float) -> np.ndarray:
    """T[k] = ceil(t_k * 2**32), k = 0..SB, as int64 (T[0] = 2**32 unused)."""
    t = 1.0
    q = 1.0 - p
    out = np.empty(SB + 1, dtype=np.int64)
    out[0] = 1 << 32
    for k in range(1, SB + 1):
        t = t * q
        out[k] = math.ceil(t * 4294967296.0)
    return out


def gap(u: int, table: np.ndarray) -> int:
    """g = #{k in 1..SB : u < T[k]} (linear count, the definition itself)."""
    return int(np.count_nonzero(u < table[1:]))


def chain_events_scalar(seed: int, instance: int, site: int, block: int,
                        p: float, K: int, table=None):
    """Events of one (site, block) stream: list of (pos in block, component)."""
    if table is None:
        table = threshold_table(p)
    key = (seed & _MASK, (seed >> 32) & _MASK)
    draws = []

    def draw(idx):
        while len(draws) <= idx:
            j = len(draws) // 4
            draws.extend(philox4x32_10((block, site, instance, j), key))
        return draws[idx]

    out = []
    d = 0
    pos = -1
    while True:
        u = draw(d)
        d += 1
        pos += gap(u, table) + 1
        if pos >= SB:
            return out
        comp = 0
        if K > 1:
            v = draw(d)
            d += 1
            comp = (v * K) >> 32
        out.append((pos, comp))


def chain_events(seed: int, instance: int, sites: np.ndarray, blocks: np.ndarray,
                 p: float, K: int, table=None):
    """All events of the streams (sites[c], blocks[c]) for every chain c.

    Same definition as chain_events_scalar, vectorised over chains.  Returns
    (chain index, pos, component) int64 arrays.
    """
    if table is None:
        table = threshold_table(p)
    sites = np.asarray(sites, dtype=np.int64)
    blocks = np.asarray(blocks, dtype=np.int64)
    n = sites.size
    key0, key1 = seed & _MASK, (seed >> 32) & _MASK
    desc = table[1:][::-1]  # ascending copy for counting u < T[k]
    pos = np.full(n, -1, dtype=np.int64)
    d = np.zeros(n, dtype=np.int64)
    active = np.ones(n, dtype=bool)
    ev_c, ev_p, ev_k = [], [], []

    def draw(idx_chains, dvals):
        words = philox4x32_10_np(blocks[idx_chains], sites[idx_chains],
                                 np.full(idx_chains.size, instance), dvals // 4,
                                 key0, key1)
        w = np.stack(words, axis=0)  # 4 x n
        return w[dvals % 4, np.arange(idx_chains.size)].astype(np.int64)

    while active.any():
        idx = np.nonzero(active)[0]
        u = draw(idx, d[idx])
        d[idx] += 1
        # number of k with u < T[k]: SB - #{k : T[k] <= u}
        g = SB - np.searchsorted(desc, u, side="right")
        pos[idx] += g + 1
        done = pos[idx] >= SB
        active[idx[done]] = False
        live = idx[~done]
        if live.size == 0:
            continue
        if K > 1:
            v = draw(live, d[live])
            d[live] += 1
            comp = (v * K) >> 32
        else:
            comp = np.zeros(live.size, dtype=np.int64)
        ev_c.append(live)
        ev_p.append(pos[live].copy())
        ev_k.append(comp)
    if not ev_c:
        e = np.zeros(0, dtype=np.int64)
        return e, e.copy(), e.copy()
    return (np.concatenate(ev_c), np.concatenate(ev_p), np.concatenate(ev_k))
