"""Flooding min-sum belief propagation on a detector error model (oracle).

The paper decodes with BP-OSD (Supplementary Note 7) but does not state BP's
equations; this is standard flooding min-sum on the DEM's check matrix H
(rows = detectors, columns = mechanisms), with prior LLRs
lambda_v = ln((1 - p_v) / p_v):

  t = 0     : e_hat = 0; if s = 0 stop (0 iterations); q_{v->c} = lambda_v
  t = 1..T  : m_{c->v} = (-1)^{s_c} * prod_{v' != v} sgn(q_{v'->c})
                         * (alpha_t(c, v) * min_{v' != v} |q_{v'->c}|)
              L_v      = lambda_v + sum_{c in N(v)} m_{c->v}   (c ascending)
              q_{v->c} = L_v - m_{c->v}
              e_hat_v  = [L_v < 0];  stop when H e_hat = s
with sgn(0) = +1 and the minimum over an empty set equal to 1e30.  alpha is a
scalar for plain BP and the per-edge, per-iteration weight w_t(c, v) for
weighted (neural) BP.

Precision: ``dtype=np.float64`` is the reference; ``dtype=np.float32`` runs the
same steps in IEEE single precision in the same order (the sum over c is
accumulated left to right), which is the precision in which the GPU decoder
takes its hard decisions and OSD orderings.

Parity: pinned against exact min-marginals on tree-shaped (repetition-code)
graphs by brute force (tests/test_oracle_decoder.py).
"""
from __future__ import annotations

import math

import numpy as np

BIG = 1e30


class Graph:
    """Edges of H in check-major order with padded per-check / per-variable views."""

    def __init__(self, H: np.ndarray):
        H = np.asarray(H, dtype=np.uint8)
        self.m, self.n = H.shape
        rows, cols = np.nonzero(H)           # row-major => check-major, v ascending
        self.ec = rows.astype(np.int64)
        self.ev = cols.astype(np.int64)
        self.E = rows.size
        deg_c = np.bincount(self.ec, minlength=self.m)
        deg_v = np.bincount(self.ev, minlength=self.n)
        self.Dc = int(deg_c.max()) if self.m else 0
        self.Dv = int(deg_v.max()) if self.n else 0
        # per-check slots: chk_edge[c, k] = edge id or -1
        self.chk_edge = -np.ones((self.m, max(self.Dc, 1)), dtype=np.int64)
        pos = np.zeros(self.m, dtype=np.int64)
        for e in range(self.E):
            c = self.ec[e]
            self.chk_edge[c, pos[c]] = e
            pos[c] += 1
        # per-variable slots in ascending check order
        self.var_edge = -np.ones((self.n, max(self.Dv, 1)), dtype=np.int64)
        order = np.lexsort((self.ec, self.ev))
        pos = np.zeros(self.n, dtype=np.int64)
        for e in order:
            v = self.ev[e]
            self.var_edge[v, pos[v]] = e
            pos[v] += 1


def prior_llr(priors: np.ndarray) -> np.ndarray:
    """lambda_v = ln((1 - p_v) / p_v), FP64, one libm call per entry."""
    return np.array([math.log((1.0 - p) / p) for p in np.asarray(priors, dtype=np.float64)],
                    dtype=np.float64)


def syndrome_of(H: np.ndarray, e: np.ndarray) -> np.ndarray:
    """H e mod 2 for e of shape [S, n] -> [S, m]."""
    return (e.astype(np.int64) @ np.asarray(H, dtype=np.int64).T) % 2 == 1


def check_to_var(g: Graph, q: np.ndarray, synd: np.ndarray, alpha, dtype):
    """Min-sum check update.  q: [S, E] -> m: [S, E]."""
    S = q.shape[0]
    big = dtype(BIG)
    slots = g.chk_edge                        # [m, Dc]
    valid = slots >= 0
    qs = np.where(valid[None], q[:, np.maximum(slots, 0)], dtype(0))
    mag = np.where(valid[None], np.abs(qs), big).astype(dtype)
    neg = (qs < 0) & valid[None]
    D = slots.shape[1]
    # minimum over the other slots: min(prefix before k, suffix after k)
    pre = np.full(mag.shape, big, dtype=dtype)
    suf = np.full(mag.shape, big, dtype=dtype)
    for k in range(1, D):
        pre[:, :, k] = np.minimum(pre[:, :, k - 1], mag[:, :, k - 1])
    for k in range(D - 2, -1, -1):
        suf[:, :, k] = np.minimum(suf[:, :, k + 1], mag[:, :, k + 1])
    others = np.minimum(pre, suf)
    par = (np.sum(neg, axis=2) % 2 == 1)[:, :, None] ^ neg   # sign of the others
    par = par ^ synd[:, :, None]
    m = np.zeros((S, g.E), dtype=dtype)
    ee = slots[valid]
    a = alpha if np.ndim(alpha) == 0 else alpha[ee][None, :]
    magn = (np.asarray(a, dtype=dtype) * others[:, valid]).astype(dtype)
    m[:, ee] = np.where(par[:, valid], -magn, magn)
    return m


def var_update(g: Graph, lam: np.ndarray, m: np.ndarray, dtype):
    """L_v = lambda_v + sum of incoming messages in ascending check order."""
    S = m.shape[0]
    L = np.broadcast_to(lam.astype(dtype), (S, g.n)).copy()
    for k in range(g.var_edge.shape[1]):
        e = g.var_edge[:, k]
        ok = e >= 0
        add = np.zeros((S, g.n), dtype=dtype)
        add[:, ok] = m[:, e[ok]]
        L = (L + add).astype(dtype)
    return L


def decode_bp(H, priors, synd, max_iter: int, alpha=1.0, weights=None,
              dtype=np.float64, graph: Graph | None = None, early_stop=True):
    """Batched min-sum.  synd: [S, m] bool.

    early_stop=False runs all max_iter iterations (the stopping rule is still
    reported in ``converged`` but does not freeze the outputs).

    weights: None or [T, E] per-edge per-iteration weights (check-major edge
    order of np.nonzero(H)).  Returns dict with e_hat [S, n] bool, llr [S, n],
    iters [S], converged [S].
    """
    g = graph or Graph(H)
    synd = np.asarray(synd, dtype=bool)
    S = synd.shape[0]
    lam = prior_llr(priors).astype(dtype)
    Hm = np.asarray(H, dtype=np.int64)
    e_hat = np.zeros((S, g.n), dtype=bool)
    llr = np.broadcast_to(lam, (S, g.n)).astype(dtype).copy()
    iters = np.zeros(S, dtype=np.int64)
    done = ~synd.any(axis=1)
    conv = done.copy()
    if not early_stop:
        done[:] = False
    q = np.broadcast_to(lam[g.ev], (S, g.E)).astype(dtype).copy()
    for t in range(1, max_iter + 1):
        act = np.nonzero(~done)[0]          # shots still iterating
        if act.size == 0:
            break
        a = dtype(alpha) if weights is None else np.asarray(weights[t - 1], dtype=dtype)
        m = check_to_var(g, q[act], synd[act], a, dtype)
        L = var_update(g, lam, m, dtype)
        q[act] = (L[:, g.ev] - m).astype(dtype)
        hard = L < 0
        ok = ((hard.astype(np.int64) @ Hm.T) % 2 == 1) == synd[act]
        ok = ok.all(axis=1)
        e_hat[act] = hard
        llr[act] = L
        iters[act] = t
        conv[act[ok]] = True
        if early_stop:
            done[act[ok]] = True
    return dict(e_hat=e_hat, llr=llr, iters=iters, converged=conv)
