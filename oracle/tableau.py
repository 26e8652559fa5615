"""Stabilizer tableau simulator (Aaronson and Gottesman, PRA 70, 052328, 2004).

A textbook CHP simulator: 2n generator rows (destabilizers then stabilizers)
plus one scratch row, each an (x | z | r) symplectic vector with sign bit.
It runs a circuit with real measurement outcomes (random ones drawn from a
caller-supplied numpy generator) and real classically-controlled Paulis, and
applies an explicit list of injected Pauli faults at noise sites instead of
sampling noise.

Used to pin the frame propagator and the circuits: in the noiseless circuit
every detector and observable must come out 0 whatever the random
measurement outcomes are; with injected faults the detector and observable
bits must equal the frame propagator's.

Parity: pinned on textbook states (Bell/GHZ correlations, deterministic vs
random outcomes) in tests/test_oracle_tableau.py.
"""
from __future__ import annotations

import numpy as np

from .circuits import NOISE_OPS
from .frame import component_paulis


class Tableau:
    def __init__(self, n: int):
        self.n = n
        self.x = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.z = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.r = np.zeros(2 * n + 1, dtype=np.uint8)
        for i in range(n):
            self.x[i, i] = 1          # destabilizer X_i
            self.z[n + i, i] = 1      # stabilizer Z_i

    # ------------------------------------------------------------- gates
    def cx(self, a, b):
        x, z = self.x, self.z
        self.r ^= x[:, a] & z[:, b] & (x[:, b] ^ z[:, a] ^ 1)
        x[:, b] ^= x[:, a]
        z[:, a] ^= z[:, b]

    def h(self, a):
        x, z = self.x, self.z
        self.r ^= x[:, a] & z[:, a]
        xa = x[:, a].copy()
        x[:, a] = z[:, a]
        z[:, a] = xa

    def pauli(self, a, p):
        """Apply Pauli p in {0:I, 1:X, 2:Y, 3:Z} to qubit a."""
        if p in (1, 2):
            self.r ^= self.z[:, a]
        if p in (2, 3):
            self.r ^= self.x[:, a]

    # ------------------------------------------------------- measurement
    @staticmethod
    def _g(x1, z1, x2, z2):
        x1 = x1.astype(np.int64); z1 = z1.astype(np.int64)
        x2 = x2.astype(np.int64); z2 = z2.astype(np.int64)
        return np.where((x1 == 0) & (z1 == 0), 0,
               np.where((x1 == 1) & (z1 == 1), z2 - x2,
               np.where((x1 == 1) & (z1 == 0), z2 * (2 * x2 - 1),
                        x2 * (1 - 2 * z2))))

    def _rowsum(self, h, i):
        tot = 2 * int(self.r[h]) + 2 * int(self.r[i]) + \
            int(self._g(self.x[i], self.z[i], self.x[h], self.z[h]).sum())
        self.r[h] = 0 if tot % 4 == 0 else 1
        self.x[h] ^= self.x[i]
        self.z[h] ^= self.z[i]

    def measure_z(self, a, rng) -> tuple[int, bool]:
        """Returns (outcome, was_random)."""
        n = self.n
        xs = np.nonzero(self.x[n:2 * n, a])[0]
        if xs.size:
            p = n + xs[0]
            for i in range(2 * n):
                if i != p and self.x[i, a]:
                    self._rowsum(i, p)
            self.x[p - n] = self.x[p]
            self.z[p - n] = self.z[p]
            self.r[p - n] = self.r[p]
            self.x[p] = 0
            self.z[p] = 0
            self.z[p, a] = 1
            out = int(rng.integers(2))
            self.r[p] = out
            return out, True
        s = 2 * n
        self.x[s] = 0
        self.z[s] = 0
        self.r[s] = 0
        for i in range(n):
            if self.x[i, a]:
                self._rowsum(s, i + n)
        return int(self.r[s]), False

    def measure_x(self, a, rng):
        self.h(a)
        out = self.measure_z(a, rng)
        self.h(a)
        return out

    def reset_z(self, a, rng):
        out, _ = self.measure_z(a, rng)
        if out:
            self.pauli(a, 1)

    def reset_x(self, a, rng):
        out, _ = self.measure_x(a, rng)
        if out:
            self.pauli(a, 3)


def run(circuit, rng, faults=()):
    """Run the circuit on a tableau.

    faults: iterable of (site, component) Pauli faults to inject (components as
    in the sampler).  Returns (detectors, observables, random_flags) as uint8
    arrays; random_flags marks measurements whose outcome was random.
    """
    by_site = {}
    for s, c in faults:
        by_site.setdefault(s, []).append(c)
    tab = Tableau(circuit.num_qubits)
    rec = []
    rnd = []
    dets = []
    obs = np.zeros(max(circuit.num_obs, 1), dtype=np.uint8)
    site = 0
    for name, arg, t in circuit.ops:
        if name == "R":
            for q in t:
                tab.reset_z(q, rng)
        elif name == "RX":
            for q in t:
                tab.reset_x(q, rng)
        elif name == "BELL_PREP":
            for a, b in zip(t[0::2], t[1::2]):
                tab.reset_z(a, rng)
                tab.reset_z(b, rng)
                tab.h(a)
                tab.cx(a, b)
        elif name == "M":
            for q in t:
                o, r = tab.measure_z(q, rng)
                rec.append(o)
                rnd.append(r)
        elif name == "MX":
            for q in t:
                o, r = tab.measure_x(q, rng)
                rec.append(o)
                rnd.append(r)
        elif name == "H":
            for q in t:
                tab.h(q)
        elif name == "CX":
            for c, tq in zip(t[0::2], t[1::2]):
                tab.cx(c, tq)
        elif name == "CXREC":
            for r, q in t:
                if rec[r]:
                    tab.pauli(q, 1)
        elif name == "CZREC":
            for r, q in t:
                if rec[r]:
                    tab.pauli(q, 3)
        elif name in NOISE_OPS:
            group = 2 if name == "DEPOLARIZE2" else 1
            g = len(t) // group
            for j in range(g):
                for comp in by_site.get(site + j, ()):
                    pa, pb = component_paulis(name, np.array([comp]))
                    tab.pauli(t[group * j], int(pa[0]))
                    if group == 2:
                        tab.pauli(t[group * j + 1], int(pb[0]))
            site += g
        elif name == "DETECTOR":
            v = 0
            for r in t:
                v ^= rec[r]
            dets.append(v)
        elif name == "OBS":
            for r in t:
                obs[arg] ^= rec[r]
        elif name == "TICK":
            pass
        else:
            raise ValueError(name)
    return (np.array(dets, dtype=np.uint8), obs[: circuit.num_obs],
            np.array(rnd, dtype=bool))
