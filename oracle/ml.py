"""Exhaustive maximum-likelihood decoding and exact expected LER (oracle).

For a detector error model with few mechanisms (N <= ~22) every error pattern
e in {0,1}^N is enumerated with probability P(e) = prod p_j^e_j (1-p_j)^(1-e_j),
syndrome s = H e and observable flips o = L e (Supplementary Note 1, syndrome
equations; the decoder picks the most likely explanation).

  LER_ML = 1 - sum_s max_o P(s, o)
  LER_D  = sum_e P(e) [decoder(H e) predicts o != L e]   for any decoder D

Used to pin the BP-OSD oracle (LER_D is what sampling must reproduce within
its statistical error, and LER_D >= LER_ML).
"""
from __future__ import annotations

import numpy as np


def enumerate_patterns(H, L, priors):
    H = np.asarray(H, dtype=np.int64)
    L = np.asarray(L, dtype=np.int64)
    p = np.asarray(priors, dtype=np.float64)
    N = H.shape[1]
    if N > 24:
        raise ValueError("too many mechanisms for exhaustive enumeration")
    idx = np.arange(1 << N, dtype=np.int64)
    E = ((idx[:, None] >> np.arange(N)) & 1).astype(np.int64)
    logp = E @ np.log(p) + (1 - E) @ np.log1p(-p)
    P = np.exp(logp)
    S = (E @ H.T) % 2
    O = (E @ L.T) % 2
    return E, P, S, O


def _key(rows):
    w = 1 << np.arange(rows.shape[1], dtype=np.int64)
    return rows @ w


def ml_ler(H, L, priors) -> float:
    _, P, S, O = enumerate_patterns(H, L, priors)
    ks, ko = _key(S), _key(O)
    best = {}
    for s, o, pr in zip(ks, ko, P):
        d = best.setdefault(int(s), {})
        d[int(o)] = d.get(int(o), 0.0) + pr
    return 1.0 - sum(max(d.values()) for d in best.values())


def expected_ler(H, L, priors, decode_fn) -> float:
    """decode_fn(synd [K, m] bool) -> predicted observables [K, k] bool."""
    E, P, S, O = enumerate_patterns(H, L, priors)
    ks = _key(S)
    uniq, first, inv = np.unique(ks, return_index=True, return_inverse=True)
    pred = np.asarray(decode_fn(S[first].astype(bool)), dtype=np.int64)
    wrong = np.any(pred[inv] != O, axis=1)
    return float(P[wrong].sum())
