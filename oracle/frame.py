"""Pauli-frame propagation and sampling (oracle).

A Pauli frame holds, per shot, the X and Z components of the difference
between the noisy run and a noiseless reference run (symplectic bits,
Supplementary Note 1).  Plain boolean arrays ``X[q, shot]``, ``Z[q, shot]``
are used: no bit packing.  Frame actions:

  R, RX, BELL_PREP : X = Z = 0 on the targets
  M  : record X[q]          MX : record Z[q]
  H  : swap X[q], Z[q]
  CX c t : X[t] ^= X[c];  Z[c] ^= Z[t]
  CXREC (r, q) : X[q] ^= record r      CZREC : Z[q] ^= record r
  DETECTOR / OBS : XOR of records

No gauge randomisation is applied: every detector and observable is a
deterministic function of the noise in these circuits (checked with the
tableau), so gauge bits cannot change any output.

Sampling noise follows ``oracle.philox``: site s of the circuit (counted in
circuit order, one per single-qubit target or per qubit pair of DEPOLARIZE2)
draws its events per 4096-shot block.  Components: DEPOLARIZE1 0->X, 1->Y,
2->Z; DEPOLARIZE2 c+1 = 4a+b with a (first qubit), b in {I,X,Y,Z}={0,1,2,3}.

Parity: pinned against the stabilizer tableau on small circuits (noiseless
all-zero detectors; identical detector bits under injected Paulis) and, for
the noise statistics, against detector marginals predicted by the detector
error model (tests/test_oracle_circuits.py, tests/test_oracle_sampler.py).
"""
from __future__ import annotations

import numpy as np

from .circuits import NOISE_OPS
from .philox import SB, chain_events, threshold_table

# Pauli index (I, X, Y, Z) -> (x bit, z bit)
PAULI_X = np.array([0, 1, 1, 0], dtype=bool)
PAULI_Z = np.array([0, 0, 1, 1], dtype=bool)
K_OF = {"X_ERROR": 1, "Z_ERROR": 1, "DEPOLARIZE1": 3, "DEPOLARIZE2": 15}


def component_paulis(name: str, comp: np.ndarray):
    """Pauli index on (first, second) target for the given components."""
    comp = np.asarray(comp)
    if name == "X_ERROR":
        return np.full(comp.shape, 1), None
    if name == "Z_ERROR":
        return np.full(comp.shape, 3), None
    if name == "DEPOLARIZE1":
        return comp + 1, None
    v = comp + 1
    return v // 4, v % 4


def propagate(circuit, num_shots: int, noise_fn):
    """Run the frame through the circuit.

    noise_fn(op_name, p, site_first, targets) -> (shot, local_site, comp)
    arrays of events to apply at that noise instruction.
    Returns (detectors [m, S] bool, observables [k, S] bool).
    """
    Q = circuit.num_qubits
    S = num_shots
    X = np.zeros((Q, S), dtype=bool)
    Z = np.zeros((Q, S), dtype=bool)
    rec = np.zeros((circuit.num_meas, S), dtype=bool)
    dets = np.zeros((circuit.num_dets, S), dtype=bool)
    obs = np.zeros((max(circuit.num_obs, 1), S), dtype=bool)
    nm = 0
    nd = 0
    site = 0
    for name, arg, t in circuit.ops:
        if name in ("R", "RX"):
            X[t] = False
            Z[t] = False
        elif name == "BELL_PREP":
            X[t] = False
            Z[t] = False
        elif name == "M":
            for q in t:
                rec[nm] = X[q]
                nm += 1
        elif name == "MX":
            for q in t:
                rec[nm] = Z[q]
                nm += 1
        elif name == "H":
            xs = X[t].copy()
            X[t] = Z[t]
            Z[t] = xs
        elif name == "CX":
            for c, tq in zip(t[0::2], t[1::2]):
                X[tq] ^= X[c]
                Z[c] ^= Z[tq]
        elif name == "CXREC":
            for r, q in t:
                X[q] ^= rec[r]
        elif name == "CZREC":
            for r, q in t:
                Z[q] ^= rec[r]
        elif name in NOISE_OPS:
            group = 2 if name == "DEPOLARIZE2" else 1
            shots, local, comp = noise_fn(name, arg, site, t)
            pa, pb = component_paulis(name, comp)
            qa = np.asarray(t[0::group], dtype=np.int64)[local]
            np.logical_xor.at(X, (qa, shots), PAULI_X[pa])
            np.logical_xor.at(Z, (qa, shots), PAULI_Z[pa])
            if group == 2:
                qb = np.asarray(t[1::2], dtype=np.int64)[local]
                np.logical_xor.at(X, (qb, shots), PAULI_X[pb])
                np.logical_xor.at(Z, (qb, shots), PAULI_Z[pb])
            site += len(t) // group
        elif name == "DETECTOR":
            v = np.zeros(S, dtype=bool)
            for r in t:
                v ^= rec[r]
            dets[nd] = v
            nd += 1
        elif name == "OBS":
            for r in t:
                obs[arg] ^= rec[r]
        elif name == "TICK":
            pass
        else:
            raise ValueError("unknown instruction " + name)
    return dets, obs[: circuit.num_obs]


def sample(circuit, seed: int, instance: int, shot_begin: int, num_shots: int):
    """Sample detector and observable bits for shots [shot_begin, +num_shots)."""
    b0 = shot_begin // SB
    b1 = (shot_begin + num_shots - 1) // SB if num_shots > 0 else b0 - 1
    blocks_range = np.arange(b0, b1 + 1, dtype=np.int64)
    tables = {}

    def noise_fn(name, p, site_first, targets):
        group = 2 if name == "DEPOLARIZE2" else 1
        g = len(targets) // group
        if p not in tables:
            tables[p] = threshold_table(p)
        sites = np.repeat(np.arange(site_first, site_first + g, dtype=np.int64),
                          blocks_range.size)
        blocks = np.tile(blocks_range, g)
        ch, pos, comp = chain_events(seed, instance, sites, blocks, p, K_OF[name],
                                     tables[p])
        shot = blocks[ch] * SB + pos - shot_begin
        keep = (shot >= 0) & (shot < num_shots)
        local = sites[ch] - site_first
        return shot[keep], local[keep], comp[keep]

    return propagate(circuit, num_shots, noise_fn)


def inject(circuit, faults):
    """Propagate explicit faults: faults = list of (site, component) per shot.

    Each shot column gets exactly the listed faults (a list per shot).
    Returns (detectors, observables) as in ``propagate``.
    """
    S = len(faults)
    by_site = {}
    for shot, fl in enumerate(faults):
        for (s, comp) in fl:
            by_site.setdefault(s, []).append((shot, comp))

    def noise_fn(name, p, site_first, targets):
        group = 2 if name == "DEPOLARIZE2" else 1
        g = len(targets) // group
        sh, lo, co = [], [], []
        for j in range(g):
            for shot, comp in by_site.get(site_first + j, ()):
                sh.append(shot)
                lo.append(j)
                co.append(comp)
        return (np.array(sh, dtype=np.int64), np.array(lo, dtype=np.int64),
                np.array(co, dtype=np.int64))

    return propagate(circuit, S, noise_fn)


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """[rows, S] bool -> [rows, ceil(S/64)] uint64, shot i = bit i%64 of word i//64."""
    rows, S = bits.shape
    W = (S + 63) // 64
    pad = np.zeros((rows, W * 64), dtype=np.uint64)
    pad[:, :S] = bits
    pad = pad.reshape(rows, W, 64)
    weights = (np.uint64(1) << np.arange(64, dtype=np.uint64))
    return (pad * weights).sum(axis=2, dtype=np.uint64)


def unpack_bits(words: np.ndarray, S: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint64)
    rows, W = words.shape
    sh = np.arange(64, dtype=np.uint64)
    bits = ((words[:, :, None] >> sh) & np.uint64(1)).astype(bool)
    return bits.reshape(rows, W * 64)[:, :S]
