"""Ebit decoherence (Methods, Decoherence) in the oracle's circuits.

Each ebit waits in memory from its generation until the non-local CNOT; both
halves then get the Pauli channel with p_X = p_Y = (1 - e^{-t/T1}) / 4 and
p_Z = (1 - e^{-t/T2}) / 2 - (1 - e^{-t/T1}) / 4, with T1 = T2 in the paper.  The
pins below evaluate those formulas and the paper's ages directly: one ebit at a
time, the j-th of n has waited t = (n - j) t_gen; in lines of f, the l-th line
has waited (n/f - l) t_gen.
"""
import math

import numpy as np
import pytest

from oracle.circuits import build_circuit, ebit_decoherence
from oracle.dem import build_dem
from oracle.frame import sample
from test_oracle_sampler import _predicted
from workloads import BB_PARAMS, NLCNOT, TELEPORT, bb, line_width, sc, with_decoherence


def _paper_channel(t, T1, T2):
    px = (1 - math.exp(-t / T1)) / 4
    py = px
    pz = (1 - math.exp(-t / T2)) / 2 - (1 - math.exp(-t / T1)) / 4
    return px, py, pz


@pytest.mark.parametrize("n,f", [(9, 1), (25, 1), (25, 5), (144, 12), (18, 3)])
def test_ages_and_channel_follow_the_paper(n, f):
    t_gen, T = 3.0e-3, 250.0                 # seconds; rate = t_gen / T
    got = ebit_decoherence(n, f, t_gen / T)
    lines = n // f
    for j in range(1, n + 1):                # generation order, 1-based as in the paper
        line = (j - 1) // f + 1
        t = (lines - line) * t_gen
        px, py, pz = _paper_channel(t, T, T)
        assert px == pytest.approx(py) and pz == pytest.approx(px, rel=1e-12, abs=1e-18)
        # DEPOLARIZE1(p) applies each of X, Y, Z with probability p / 3
        assert got[j - 1] == pytest.approx(px + py + pz, rel=1e-12, abs=1e-18)
    assert got[-1] == 0.0                    # the newest ebits have not waited
    assert got[0] == max(got)


def test_line_width_rule():
    assert line_width(sc(7)) == 7
    # BB codes: the divisor of n closest to d
    expect = {"bb18": 3, "bb36": 6, "bb54": 9, "bb90": 10, "bb144": 12}
    for name, f in expect.items():
        n, _, d = BB_PARAMS[name]
        assert n % f == 0
        assert line_width(bb(name)) == f


def test_no_decoherence_leaves_the_circuit_unchanged():
    spec = sc(3, NLCNOT, 3, 3, 1e-3, 1e-2)
    base = build_circuit(spec).text()
    assert build_circuit(with_decoherence(spec, 0.0, False)).text() == base
    assert build_circuit(with_decoherence(spec, 0.0, True)).text() == base


@pytest.mark.parametrize("lines", [False, True], ids=["one-at-a-time", "lines"])
def test_decoherence_instructions(lines):
    spec = with_decoherence(sc(3, NLCNOT, 2, 2, 1e-3, 1e-2), 0.05, lines)
    c = build_circuit(spec)
    i = next(k for k, (name, arg, t) in enumerate(c.ops) if name == "DEPOLARIZE2" and arg == spec.p_ebit)
    pairs = c.ops[i][2]
    ea, eb = pairs[0::2], pairs[1::2]
    dec = []
    for name, arg, t in c.ops[i + 1:]:
        if name != "DEPOLARIZE1":
            break
        dec.append((arg, t))
    expect = [(p, [ea[k], eb[k]]) for k, p in enumerate(ebit_decoherence(9, spec.ebit_per_step, 0.05)) if p > 0]
    assert dec == expect
    assert len(dec) == (8 if not lines else 6)


def test_detector_marginals_with_decoherence_match_dem():
    """Sampled detector and observable marginals agree with the DEM closed form
    on a circuit whose oldest ebits decohere strongly."""
    spec = with_decoherence(sc(3, NLCNOT, 2, 2, 2e-3, 1e-2), 0.1, False)
    c = build_circuit(spec)
    dem = build_dem(c)
    N = 3 * 4096 + 77
    dets, obs = sample(c, seed=9, instance=0, shot_begin=0, num_shots=N)
    pd, po = _predicted(dem)
    z = 4.5
    for i in range(dem.num_dets):
        assert abs(dets[i].mean() - pd[i]) < z * np.sqrt(pd[i] * (1 - pd[i]) / N)
    for o in range(dem.num_obs):
        assert abs(obs[o].mean() - po[o]) < z * np.sqrt(po[o] * (1 - po[o]) / N)
    # the decoherence is visible: the observables flip more often than without it
    _, po0 = _predicted(build_dem(build_circuit(sc(3, NLCNOT, 2, 2, 2e-3, 1e-2))))
    assert (po > po0 + 1e-3).any()
