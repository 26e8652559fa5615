"""OSD-0 and the full BP-OSD decode (oracle).

OSD-0 (ordered statistics decoding of order zero; Panteleev and Kalachev 2021,
Roffe et al. 2020 - the "BP-OSD" the paper names in Supplementary Note 7):

1. order the columns of H by (posterior LLR L_v ascending, v ascending), i.e.
   least reliable "no error" first;
2. scan the columns in that order and keep a column when it is linearly
   independent (over GF(2)) of the columns kept so far; stop once rank(H)
   columns are kept (the information set S);
3. solve H_S e_S = s on the kept columns (unique, H_S has full column rank)
   and set e = 0 elsewhere.

Independence is tested with a textbook XOR basis keyed by the highest set
bit, on columns stored as Python integers (bit r = row r).  Each basis vector
carries the set of kept columns it is the sum of, which yields e_S once s is
reduced to zero.

BP-OSD decode: BP first; if BP converged its hard decision is the answer,
otherwise OSD-0 runs on BP's final posterior LLRs.

Parity: H e = s is checked on every call; the solution is cross-checked with
a dense Gauss-Jordan solve on the same column set, and on tiny codes with
exhaustive search (tests/test_oracle_decoder.py).
"""
from __future__ import annotations

import numpy as np

from .bp import Graph, decode_bp
from .codes import rank as gf2_rank


def column_ints(H: np.ndarray):
    H = np.asarray(H, dtype=np.uint8)
    cols = []
    for v in range(H.shape[1]):
        x = 0
        for r in np.nonzero(H[:, v])[0]:
            x |= 1 << int(r)
        cols.append(x)
    return cols


def vec_int(bits) -> int:
    x = 0
    for r in np.nonzero(np.asarray(bits))[0]:
        x |= 1 << int(r)
    return x


def osd0(cols, rank_h: int, synd_bits, llr):
    """Returns (e_hat bool[n], kept column list, in_span flag)."""
    n = len(cols)
    llr = np.asarray(llr)
    order = np.lexsort((np.arange(n), llr))   # primary key llr, then index
    basis = {}      # highest bit -> (vector, combination over kept indices)
    kept = []
    for v in order:
        if len(kept) == rank_h:
            break
        vec = cols[int(v)]
        combo = 1 << len(kept)
        while vec:
            hb = vec.bit_length() - 1
            if hb not in basis:
                break
            bv, bc = basis[hb]
            vec ^= bv
            combo ^= bc
        if vec:
            basis[vec.bit_length() - 1] = (vec, combo)
            kept.append(int(v))
    s = vec_int(synd_bits)
    combo = 0
    while s:
        hb = s.bit_length() - 1
        if hb not in basis:
            break
        bv, bc = basis[hb]
        s ^= bv
        combo ^= bc
    e = np.zeros(n, dtype=bool)
    for i, v in enumerate(kept):
        if (combo >> i) & 1:
            e[v] = True
    return e, kept, s == 0


def osd_cs(cols, rank_h: int, synd_bits, llr, order: int):
    """OSD-CS of order lambda (Roffe, White, Burton, Campbell 2020, "combination
    sweep"; the higher-order OSD the paper's BP-OSD runs with order 7).

    The information set S is the first rank(H) GF(2)-independent columns in
    (L_v, v) order, and T the other columns in that order.  Candidates: the
    OSD-0 solution (e_T = 0), then e_T of weight one over all of T, then e_T of
    weight two over the first `order` columns of T (pairs a < b in order); for
    each, e_S solves H_S e_S = s + H_T e_T.  The one with the least soft weight
    sum_{e_i = 1} L_i wins; the soft weight is summed in FP32, over S in order of
    selection and then the flipped T columns in order, and a later candidate
    must be strictly lighter.  Returns (e_hat bool[n], in_span flag).
    """
    n = len(cols)
    llr = np.asarray(llr, dtype=np.float32)
    order_v = np.lexsort((np.arange(n), llr))
    basis = {}
    kept, rest = [], []
    for v in order_v:
        v = int(v)
        if len(kept) < rank_h:
            vec, combo = cols[v], 1 << len(kept)
            while vec:
                hb = vec.bit_length() - 1
                if hb not in basis:
                    break
                bv, bc = basis[hb]
                vec ^= bv
                combo ^= bc
            if vec:
                basis[vec.bit_length() - 1] = (vec, combo)
                kept.append(v)
                continue
        rest.append(v)

    def rep(x):
        """Kept columns whose sum is the column vector x (x must be in the span)."""
        combo = 0
        while x:
            hb = x.bit_length() - 1
            if hb not in basis:
                return None
            bv, bc = basis[hb]
            x ^= bv
            combo ^= bc
        return combo

    e_s = rep(vec_int(synd_bits))
    if e_s is None:
        e, _, _ = osd0(cols, rank_h, synd_bits, llr)
        return e, False

    def weight(combo, extra):
        c = np.float32(0.0)
        for i in range(len(kept)):
            if (combo >> i) & 1:
                c = np.float32(c + llr[kept[i]])
        for j in extra:
            c = np.float32(c + llr[j])
        return c

    best = (weight(e_s, []), e_s, [])
    for j in rest:
        r = rep(cols[j])
        cand = (weight(e_s ^ r, [j]), e_s ^ r, [j])
        if cand[0] < best[0]:
            best = cand
    head = rest[:order]
    for a in range(len(head)):
        for b in range(a + 1, len(head)):
            r = rep(cols[head[a]]) ^ rep(cols[head[b]])
            cand = (weight(e_s ^ r, [head[a], head[b]]), e_s ^ r, [head[a], head[b]])
            if cand[0] < best[0]:
                best = cand
    e = np.zeros(n, dtype=bool)
    for i, v in enumerate(kept):
        if (best[1] >> i) & 1:
            e[v] = True
    for j in best[2]:
        e[j] = True
    return e, True


class Decoder:
    """BP-OSD over one DEM (H, priors, L)."""

    def __init__(self, H, priors, L, max_iter=30, alpha=1.0, weights=None,
                 dtype=np.float64, use_osd=True, osd_order=0):
        self.H = np.asarray(H, dtype=np.uint8)
        self.priors = np.asarray(priors, dtype=np.float64)
        self.L = np.asarray(L, dtype=np.uint8)
        self.max_iter = max_iter
        self.alpha = alpha
        self.weights = weights
        self.dtype = dtype
        self.use_osd = use_osd
        self.osd_order = osd_order
        self.graph = Graph(self.H)
        self.cols = column_ints(self.H)
        self.rank = gf2_rank(self.H)

    def decode(self, synd: np.ndarray, chunk=256):
        synd = np.asarray(synd, dtype=bool)
        S = synd.shape[0]
        out_e = np.zeros((S, self.H.shape[1]), dtype=bool)
        out = dict(iters=np.zeros(S, np.int64), converged=np.zeros(S, bool),
                   osd=np.zeros(S, bool), in_span=np.ones(S, bool),
                   llr=np.zeros((S, self.H.shape[1]), dtype=self.dtype))
        for a in range(0, S, chunk):
            r = decode_bp(self.H, self.priors, synd[a:a + chunk], self.max_iter,
                          alpha=self.alpha, weights=self.weights, dtype=self.dtype,
                          graph=self.graph)
            out_e[a:a + chunk] = r["e_hat"]
            out["iters"][a:a + chunk] = r["iters"]
            out["converged"][a:a + chunk] = r["converged"]
            out["llr"][a:a + chunk] = r["llr"]
            if not self.use_osd:
                continue
            for i in np.nonzero(~r["converged"])[0]:
                if self.osd_order > 0:
                    e, ok = osd_cs(self.cols, self.rank, synd[a + i], r["llr"][i], self.osd_order)
                else:
                    e, _, ok = osd0(self.cols, self.rank, synd[a + i], r["llr"][i])
                out_e[a + i] = e
                out["osd"][a + i] = True
                out["in_span"][a + i] = ok
        out["e_hat"] = out_e
        out["pred_obs"] = (out_e.astype(np.int64) @ self.L.T.astype(np.int64)) % 2 == 1
        return out


def logical_errors(pred_obs: np.ndarray, obs: np.ndarray) -> np.ndarray:
    """A shot fails iff any observable prediction differs (Methods, Decoding)."""
    return np.any(np.asarray(pred_obs, bool) != np.asarray(obs, bool), axis=1)


def ler_stats(n_err: int, n_shots: int):
    """LER and its binomial standard deviation sqrt(p(1-p)/N)."""
    p = n_err / n_shots if n_shots else 0.0
    sigma = (p * (1.0 - p) / n_shots) ** 0.5 if n_shots else 0.0
    return p, sigma
