"""Detector error model by single-fault injection (oracle).

For every noise site and every Pauli component of its channel, one fault is
propagated from that site to the end of the circuit with the frame
propagator, and the flipped detectors and observables are recorded (the
"error mechanisms" of Methods, Decoding; Table III caption: one column per
distinct mechanism).

Each channel is replaced by independent mechanisms with the same output
distribution:
  X_ERROR(p), Z_ERROR(p) : one mechanism, probability p
  DEPOLARIZE1(p)         : 3 mechanisms, q1 = (1 - sqrt(1 - 4p/3)) / 2
  DEPOLARIZE2(p)         : 15 mechanisms, q2 = (1 - (1 - 16p/15)^(1/8)) / 2
(then q1(1-q1) = p/3 and (1 - (1-2 q2)^8)/16 = p/15).  The eighth root is
taken as three nested square roots so that it is correctly rounded at each
step.

Mechanisms with identical (detectors, observables) symptoms are merged in
circuit order (site, then component) with p <- pa + pb - 2 pa pb.  Empty
symptoms are dropped.  Symptoms with observables but no detectors are
undetectable logical errors: they are counted and excluded.  Columns are
sorted by (sorted detector list, observable mask) lexicographically.

Parity: pinned by brute-force circuit distance of the d=3 surface-code
operations (Table I), by the detector marginals of sampled shots, and by exact
enumeration: the independent mechanisms of each channel reproduce the
channel's Pauli distribution, the merge rule equals the XOR of two Bernoulli
variables, and the DEM of one-channel circuits gives the exact joint detector
distribution (tests/test_oracle_circuits.py, tests/test_oracle_sampler.py,
tests/test_oracle_pins.py).
"""
from __future__ import annotations

import math

import numpy as np

from .circuits import NOISE_OPS
from .frame import K_OF, propagate


def component_prob(name: str, p: float) -> float:
    if name in ("X_ERROR", "Z_ERROR"):
        return p
    if name == "DEPOLARIZE1":
        return (1.0 - math.sqrt(1.0 - 4.0 * p / 3.0)) / 2.0
    if name == "DEPOLARIZE2":
        return (1.0 - math.sqrt(math.sqrt(math.sqrt(1.0 - 16.0 * p / 15.0)))) / 2.0
    raise ValueError(name)


def merge_prob(pa: float, pb: float) -> float:
    """Probability that exactly one of two independent events (probabilities pa,
    pb) happens: two mechanisms with the same symptom flip it together iff an odd
    number of them fires."""
    return pa + pb - 2.0 * pa * pb


def site_table(circuit):
    """Per site: (channel name, p) in circuit order."""
    out = []
    for name, arg, t in circuit.ops:
        if name in NOISE_OPS:
            g = len(t) // (2 if name == "DEPOLARIZE2" else 1)
            out += [(name, arg)] * g
    return out


def fault_symptoms(circuit, sites: np.ndarray, comps: np.ndarray):
    """Detector/observable bits of single faults (one fault per column)."""
    sites = np.asarray(sites, dtype=np.int64)
    comps = np.asarray(comps, dtype=np.int64)
    order = np.argsort(sites, kind="stable")
    s_sorted = sites[order]

    def noise_fn(name, p, site_first, targets):
        g = len(targets) // (2 if name == "DEPOLARIZE2" else 1)
        lo = np.searchsorted(s_sorted, site_first, side="left")
        hi = np.searchsorted(s_sorted, site_first + g, side="left")
        idx = order[lo:hi]
        return idx, sites[idx] - site_first, comps[idx]

    return propagate(circuit, sites.size, noise_fn)


class DEM:
    """Columns (detector tuple, observable mask, probability), canonical order."""

    def __init__(self, num_dets, num_obs, cols, undetectable):
        self.num_dets = num_dets
        self.num_obs = num_obs
        self.cols = cols
        self.undetectable = undetectable  # list of (obs mask, p) excluded

    @property
    def num_cols(self):
        return len(self.cols)

    def priors(self):
        return np.array([c[2] for c in self.cols], dtype=np.float64)

    def H(self) -> np.ndarray:
        h = np.zeros((self.num_dets, self.num_cols), dtype=np.uint8)
        for j, (dets, _, _) in enumerate(self.cols):
            h[list(dets), j] = 1
        return h

    def L(self) -> np.ndarray:
        l = np.zeros((self.num_obs, self.num_cols), dtype=np.uint8)
        for j, (_, om, _) in enumerate(self.cols):
            for o in range(self.num_obs):
                if (om >> o) & 1:
                    l[o, j] = 1
        return l


def build_dem(circuit, chunk: int = 65536) -> DEM:
    table = site_table(circuit)
    fs, fc, fp = [], [], []
    for s, (name, p) in enumerate(table):
        q = component_prob(name, p)
        for comp in range(K_OF[name]):
            fs.append(s)
            fc.append(comp)
            fp.append(q)
    fs = np.array(fs, dtype=np.int64)
    fc = np.array(fc, dtype=np.int64)
    merged = {}   # symptom -> probability, insertion in circuit order
    for a in range(0, fs.size, chunk):
        dets, obs = fault_symptoms(circuit, fs[a:a + chunk], fc[a:a + chunk])
        for j in range(dets.shape[1]):
            d = tuple(np.nonzero(dets[:, j])[0].tolist())
            om = 0
            for o in np.nonzero(obs[:, j])[0]:
                om |= 1 << int(o)
            key = (d, om)
            q = fp[a + j]
            if key in merged:
                merged[key] = merge_prob(merged[key], q)
            else:
                merged[key] = q
    cols = []
    undetectable = []
    for (d, om), p in merged.items():
        if len(d) == 0:
            if om:
                undetectable.append((om, p))
            continue
        cols.append((d, om, p))
    cols.sort(key=lambda c: (list(c[0]), c[1]))
    return DEM(circuit.num_dets, circuit.num_obs, cols, undetectable)
