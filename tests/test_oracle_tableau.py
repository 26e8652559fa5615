"""Textbook pins of the CHP tableau (oracle.tableau)."""
import numpy as np

from oracle.tableau import Tableau


def test_single_qubit_states():
    rng = np.random.default_rng(0)
    t = Tableau(1)
    assert t.measure_z(0, rng) == (0, False)        # |0>
    t.pauli(0, 1)
    assert t.measure_z(0, rng) == (1, False)        # X|0> = |1>
    t = Tableau(1)
    t.h(0)
    assert t.measure_x(0, rng) == (0, False)        # |+> in the X basis
    out, rnd = t.measure_z(0, rng)
    assert rnd                                      # |+> in the Z basis is random
    assert t.measure_z(0, rng) == (out, False)      # repeated measurement agrees


def test_bell_and_ghz_correlations():
    for seed in range(10):
        rng = np.random.default_rng(seed)
        t = Tableau(3)
        t.h(0)
        t.cx(0, 1)
        t.cx(1, 2)
        a, ra = t.measure_z(0, rng)
        b, rb = t.measure_z(1, rng)
        c, rc = t.measure_z(2, rng)
        assert ra and not rb and not rc
        assert a == b == c
        t = Tableau(2)
        t.h(0)
        t.cx(0, 1)
        x0, r0 = t.measure_x(0, rng)
        x1, r1 = t.measure_x(1, rng)
        assert r0 and not r1 and x0 == x1           # XX = +1 on |Phi+>


def test_phase_tracking():
    rng = np.random.default_rng(1)
    t = Tableau(2)
    t.h(0)
    t.cx(0, 1)
    t.pauli(1, 3)                                   # Z on one half: |Phi->
    x0, _ = t.measure_x(0, rng)
    x1, _ = t.measure_x(1, rng)
    assert x0 ^ x1 == 1
    t = Tableau(1)
    t.pauli(0, 2)                                   # Y|0> ~ |1>
    assert t.measure_z(0, rng)[0] == 1
