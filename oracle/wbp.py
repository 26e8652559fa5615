"""Weighted (neural) min-sum BP: unrolled forward and its reverse-mode gradient (oracle).

Weighted min-sum replaces the scalar scaling of plain min-sum by a learned
weight per edge and per iteration, w_t(c, v), and runs a fixed number T of
flooding iterations with no early stop (the paper's decoder is BP-OSD,
Supplementary Note 7; the learned weights are this library's addition):

  q0_{v->c} = lambda_v
  m_t(c, v) = w_t(c, v) * sigma_t(c, v) * mu_t(c, v)
      sigma_t(c, v) = (-1)^{s_c} prod_{v' != v} sgn(q_{t-1}(v' -> c))
      mu_t(c, v)    = min_{v' != v} |q_{t-1}(v' -> c)|          (1e30 if empty)
  L_t(v) = lambda_v + sum_c m_t(c, v)
  q_t(v -> c) = L_t(v) - m_t(c, v)

Reverse mode, given G_t(v) = dLoss/dL_t(v) for t = 1..T:
  gq_T = 0
  for t = T..1:
      gL_t(v)   = G_t(v) + sum_c gq_t(v -> c)
      gm_t(c,v) = gL_t(v) - gq_t(v -> c)
      dLoss/dw_t(c,v) = gm_t(c,v) * sigma_t(c,v) * mu_t(c,v)      (0 where mu = 1e30)
      gq_{t-1}(v* -> c) += gm_t(c,v) * w_t(c,v) * sigma_t(c,v) * sgn(q_{t-1}(v* -> c))
          with v* the lowest-index edge attaining mu_t(c, v) (signs carry no gradient;
          the 1e30 of an empty minimum carries none either)

Everything is explicit per edge, in FP64 unless ``dtype`` says otherwise.
Edges are the nonzeros of H in row-major (check-major) order.

Parity: the gradient is pinned by central finite differences of the forward
(tests/test_oracle_wbp.py).
"""
from __future__ import annotations

import numpy as np

from .bp import BIG, Graph, prior_llr


def forward(H, priors, synd, weights, dtype=np.float64, graph: Graph | None = None):
    """synd [S, m] bool, weights [T, E].  Returns dict with L [T, S, n] and the
    per-iteration quantities the backward pass needs (q_{t-1}, mu, argmin, sigma)."""
    g = graph or Graph(H)
    synd = np.asarray(synd, dtype=bool)
    S = synd.shape[0]
    T = weights.shape[0]
    lam = prior_llr(priors).astype(dtype)
    W = np.asarray(weights, dtype=dtype)
    q = np.broadcast_to(lam[g.ev], (S, g.E)).astype(dtype).copy()
    Ls = np.zeros((T, S, g.n), dtype=dtype)
    saved = []
    rows = [g.chk_edge[c][g.chk_edge[c] >= 0] for c in range(g.m)]
    for t in range(T):
        mu = np.full((S, g.E), dtype(BIG), dtype=dtype)
        amin = -np.ones((S, g.E), dtype=np.int64)      # edge attaining mu (lowest index)
        sigma = np.ones((S, g.E), dtype=dtype)
        for c, es in enumerate(rows):
            aq = np.abs(q[:, es])
            neg = q[:, es] < 0
            for k, e in enumerate(es):
                others = [j for j in range(len(es)) if j != k]
                if others:
                    sub = aq[:, others]
                    pick = np.argmin(sub, axis=1)          # first (lowest index) minimum
                    mu[:, e] = sub[np.arange(S), pick]
                    amin[:, e] = es[np.array(others)[pick]]
                    par = (neg[:, others].sum(axis=1) % 2 == 1) ^ synd[:, c]
                else:
                    par = synd[:, c].copy()
                sigma[:, e] = np.where(par, -1.0, 1.0)
        m = (W[t][None, :] * mu).astype(dtype) * sigma
        m = m.astype(dtype)
        L = np.broadcast_to(lam, (S, g.n)).astype(dtype).copy()
        for k in range(g.var_edge.shape[1]):
            e = g.var_edge[:, k]
            ok = e >= 0
            add = np.zeros((S, g.n), dtype=dtype)
            add[:, ok] = m[:, e[ok]]
            L = (L + add).astype(dtype)
        saved.append(dict(q_prev=q.copy(), mu=mu, amin=amin, sigma=sigma, m=m))
        q = (L[:, g.ev] - m).astype(dtype)
        Ls[t] = L
    return dict(L=Ls, saved=saved, graph=g, weights=W)


def backward(fwd, G):
    """G [T, S, n] = dLoss/dL_t.  Returns dLoss/dw as [T, E] (FP64)."""
    g = fwd["graph"]
    W = np.asarray(fwd["weights"], dtype=np.float64)
    T, S, n = G.shape
    gW = np.zeros((T, g.E), dtype=np.float64)
    gq = np.zeros((S, g.E), dtype=np.float64)
    for t in range(T - 1, -1, -1):
        sv = fwd["saved"][t]
        gL = np.asarray(G[t], dtype=np.float64).copy()
        np.add.at(gL, (slice(None), g.ev), gq)                     # sum over checks of gq_t
        gm = gL[:, g.ev] - gq
        mu = sv["mu"].astype(np.float64)
        sigma = sv["sigma"].astype(np.float64)
        finite = mu < BIG / 2
        gW[t] = np.sum(np.where(finite, gm * sigma * mu, 0.0), axis=0)
        gq_prev = np.zeros((S, g.E), dtype=np.float64)
        q_prev = sv["q_prev"].astype(np.float64)
        contrib = np.where(finite, gm * W[t][None, :] * sigma, 0.0)
        for s in range(S):
            tgt = sv["amin"][s]
            ok = tgt >= 0
            sgn = np.where(q_prev[s, tgt[ok]] < 0, -1.0, 1.0)
            np.add.at(gq_prev[s], tgt[ok], contrib[s, ok] * sgn)
        gq = gq_prev
    return gW
