"""Quantum codes: rotated surface code and bivariate-bicycle codes (oracle).

* Rotated surface code [[d^2, 1, d]] (Supplementary Note 2): d x d data
  qubits; weight-4 bulk plaquettes and weight-2 boundary plaquettes of X and
  Z type.  Layout used here: plaquette (i, j), i, j in -1..d-1, has corners
  NW=(i,j), NE=(i,j+1), SW=(i+1,j), SE=(i+1,j+1) (those inside the grid);
  its type is X when i+j is even, else Z; bulk plaquettes are all kept, the
  top/bottom boundary keeps X plaquettes, the left/right boundary keeps Z
  plaquettes.  Z_L = Z on data row 0 (weight d).
* Bivariate-bicycle codes (Supplementary Note 3, Table IV):
  x = S_l (x) I_m, y = I_l (x) S_m with S_j the cyclic shift
  S_j[r, (r+1) mod j] = 1; A = a(x, y), B = b(x, y); H_X = [A|B],
  H_Z = [B^T|A^T].  Data qubit c < lm is "left" qubit (i, j) = divmod(c, m);
  c >= lm is the right qubit c - lm.
* Logical Z basis for BB codes (the paper does not fix one): the rows of the
  reduced row echelon form (RREF) of ker(H_X), taken in order, keeping each row
  that is independent of rowspace(H_Z) and of the rows already kept.  The RREF
  of a subspace is unique, so this basis is a definition, not an accident of
  implementation.

Parity: pinned by k from GF(2) ranks against the names in Table IV, by the CSS
condition H_X H_Z^T = 0, by row/column weights, and by brute-force code
distances of the small codes (tests/test_oracle_codes.py).
"""
from __future__ import annotations

import numpy as np

from workloads import BB_CODES, CircuitSpec, SC


# --------------------------------------------------------------------- GF(2)
def rref(mat: np.ndarray):
    """Reduced row echelon form over GF(2).  Returns (R, pivot columns)."""
    a = (np.array(mat, dtype=np.uint8) & 1).copy()
    rows, cols = a.shape
    piv = []
    r = 0
    for c in range(cols):
        if r >= rows:
            break
        nz = np.nonzero(a[r:, c])[0]
        if nz.size == 0:
            continue
        k = r + nz[0]
        if k != r:
            a[[r, k]] = a[[k, r]]
        for i in range(rows):
            if i != r and a[i, c]:
                a[i] ^= a[r]
        piv.append(c)
        r += 1
    return a[:r], piv


def rank(mat: np.ndarray) -> int:
    return len(rref(mat)[1])


def kernel(mat: np.ndarray) -> np.ndarray:
    """A basis (as rows) of {v : mat v = 0}, in RREF."""
    mat = np.array(mat, dtype=np.uint8)
    n = mat.shape[1]
    r, piv = rref(mat)
    free = [c for c in range(n) if c not in set(piv)]
    basis = []
    for f in free:
        v = np.zeros(n, dtype=np.uint8)
        v[f] = 1
        for row, pc in zip(r, piv):
            if row[f]:
                v[pc] = 1
        basis.append(v)
    if not basis:
        return np.zeros((0, n), dtype=np.uint8)
    return rref(np.array(basis))[0]


# ------------------------------------------------------------ code objects
class Code:
    """A CSS code block with its syndrome-extraction schedule.

    Attributes
      n, k         : parameters
      hx, hz       : check matrices (uint8)
      lz           : logical Z operators (k x n uint8)
      x_sched      : list of layers; each layer is a list of (check, data)
      z_sched      : same for Z checks
      sched_layers : number of CX layers per round (both types share layers)
    """


def surface_code(d: int) -> Code:
    c = Code()
    c.kind = SC
    c.d = d
    n = d * d
    c.n = n
    xs, zs = [], []  # list of corner lists [NW, NE, SW, SE], None if absent
    for i in range(-1, d):
        for j in range(-1, d):
            bulk = 0 <= i <= d - 2 and 0 <= j <= d - 2
            is_x = (i + j) % 2 == 0
            top_bottom = (i == -1 or i == d - 1) and 0 <= j <= d - 2
            left_right = (j == -1 or j == d - 1) and 0 <= i <= d - 2
            keep = bulk or (top_bottom and is_x) or (left_right and not is_x)
            if not keep:
                continue
            corners = []
            for (a, b) in ((i, j), (i, j + 1), (i + 1, j), (i + 1, j + 1)):
                corners.append(a * d + b if (0 <= a < d and 0 <= b < d) else None)
            (xs if is_x else zs).append(corners)
    c.hx = np.zeros((len(xs), n), dtype=np.uint8)
    c.hz = np.zeros((len(zs), n), dtype=np.uint8)
    for r, cs in enumerate(xs):
        for q in cs:
            if q is not None:
                c.hx[r, q] = 1
    for r, cs in enumerate(zs):
        for q in cs:
            if q is not None:
                c.hz[r, q] = 1
    # hook-avoiding order: X checks NW, NE, SW, SE; Z checks NW, SW, NE, SE
    x_order = (0, 1, 2, 3)
    z_order = (0, 2, 1, 3)
    c.x_sched = [[(r, cs[x_order[t]]) for r, cs in enumerate(xs) if cs[x_order[t]] is not None]
                 for t in range(4)]
    c.z_sched = [[(r, cs[z_order[t]]) for r, cs in enumerate(zs) if cs[z_order[t]] is not None]
                 for t in range(4)]
    c.sched_layers = 4
    c.interleaved = True  # X and Z layers run in the same 4 time steps
    lz = np.zeros((1, n), dtype=np.uint8)
    lz[0, :d] = 1  # Z on data row 0
    c.lz = lz
    c.k = 1
    return c


# BB syndrome schedule: the term each X (Z) check applies at each of the 7 CX
# steps of a round (-1: idle).  This is the depth-optimised interleaved cycle of
# the bivariate-bicycle memory experiments the paper builds its BB circuits on
# (Methods, "Simulation").
BB_X_STEPS = (-1, 1, 4, 3, 5, 0, 2)
BB_Z_STEPS = (3, 5, 0, 1, 2, 4, -1)


def _mono_perm(l: int, m: int, a: int, b: int) -> np.ndarray:
    """Column index of the single 1 in each row of x^a y^b (length lm)."""
    r = np.arange(l * m)
    i, j = r // m, r % m
    return ((i + a) % l) * m + (j + b) % m


def _perm_matrix(perm: np.ndarray) -> np.ndarray:
    n = perm.size
    mat = np.zeros((n, n), dtype=np.uint8)
    mat[np.arange(n), perm] = 1
    return mat


def bb_code(name: str) -> Code:
    l, m, a_terms, b_terms = BB_CODES[name]
    c = Code()
    c.kind = "bb"
    c.name = name
    h = l * m
    n = 2 * h
    c.n = n
    pa = [_mono_perm(l, m, *t) for t in a_terms]
    pb = [_mono_perm(l, m, *t) for t in b_terms]
    A = np.zeros((h, h), dtype=np.uint8)
    B = np.zeros((h, h), dtype=np.uint8)
    for p in pa:
        A ^= _perm_matrix(p)
    for p in pb:
        B ^= _perm_matrix(p)
    c.A, c.B = A, B
    c.hx = np.concatenate([A, B], axis=1)
    c.hz = np.concatenate([B.T, A.T], axis=1)
    # Interleaved depth-7 schedule (R16): step t runs one term of every X check
    # and one term of every Z check on the other half of the data.  X terms
    # 0-2 are A_1..A_3 (left data), 3-5 are B_1..B_3 (right data); Z terms 0-2
    # are B_1^T..B_3^T (left data), 3-5 are A_1^T..A_3^T (right data).
    inv = lambda p: np.argsort(p)
    rows = np.arange(h)
    x_term = [[(int(r), int(p[r])) for r in rows] for p in pa] + \
             [[(int(r), h + int(p[r])) for r in rows] for p in pb]
    z_term = [[(int(r), int(inv(p)[r])) for r in rows] for p in pb] + \
             [[(int(r), h + int(inv(p)[r])) for r in rows] for p in pa]
    c.x_sched = [x_term[t] if t >= 0 else [] for t in BB_X_STEPS]
    c.z_sched = [z_term[t] if t >= 0 else [] for t in BB_Z_STEPS]
    c.sched_layers = len(BB_X_STEPS)
    c.interleaved = True
    c.k = n - rank(c.hx) - rank(c.hz)
    c.lz = logical_z_basis(c.hx, c.hz, c.k)
    return c


def logical_z_basis(hx: np.ndarray, hz: np.ndarray, k: int) -> np.ndarray:
    """RREF rows of ker(H_X), kept greedily when independent of rowspace(H_Z)."""
    ker = kernel(hx)
    kept = []
    base = rank(hz)
    for v in ker:
        trial = np.vstack([hz] + kept + [v[None, :]])
        if rank(trial) > base + len(kept):
            kept.append(v[None, :])
        if len(kept) == k:
            break
    return np.vstack(kept) if kept else np.zeros((0, hx.shape[1]), dtype=np.uint8)


def make_code(spec: CircuitSpec) -> Code:
    if spec.code == SC:
        return surface_code(spec.d)
    return bb_code(spec.bb)
