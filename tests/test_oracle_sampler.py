"""Pin the sampled noise statistics against the detector error model."""
import numpy as np
import pytest

from oracle.circuits import build_circuit
from oracle.dem import build_dem
from oracle.frame import pack_bits, sample, unpack_bits
from workloads import MEMORY, NLCNOT, sc


def _predicted(dem):
    """P(D_i = 1) = (1 - prod_{j ni i} (1 - 2 p_j)) / 2 for independent mechanisms."""
    prod = np.ones(dem.num_dets)
    oprod = np.ones(dem.num_obs)
    for dets, om, p in dem.cols:
        for i in dets:
            prod[i] *= 1 - 2 * p
        for o in range(dem.num_obs):
            if (om >> o) & 1:
                oprod[o] *= 1 - 2 * p
    return (1 - prod) / 2, (1 - oprod) / 2


@pytest.mark.parametrize("spec", [sc(3, MEMORY, 3, 0, 1e-2), sc(3, NLCNOT, 2, 2, 5e-3, 2e-2)],
                         ids=["sc3-memory", "sc3-nlcnot"])
def test_detector_marginals_match_dem(spec):
    c = build_circuit(spec)
    dem = build_dem(c)
    N = 3 * 4096 + 123                       # several blocks and a ragged tail
    dets, obs = sample(c, seed=5, instance=1, shot_begin=777, num_shots=N)
    pd, po = _predicted(dem)
    z = 4.5                                   # Bonferroni over ~70 detectors
    for i in range(dem.num_dets):
        sig = np.sqrt(pd[i] * (1 - pd[i]) / N)
        assert abs(dets[i].mean() - pd[i]) < z * sig
    for o in range(dem.num_obs):
        sig = np.sqrt(po[o] * (1 - po[o]) / N)
        assert abs(obs[o].mean() - po[o]) < z * sig


def test_shot_ranges_compose():
    """Resumability: [0, a) + [a, N) equals [0, N) bit for bit."""
    c = build_circuit(sc(3, MEMORY, 2, 0, 2e-2))
    N, a = 9000, 4100
    d_all, o_all = sample(c, 3, 0, 0, N)
    d1, o1 = sample(c, 3, 0, 0, a)
    d2, o2 = sample(c, 3, 0, a, N - a)
    assert (np.concatenate([d1, d2], axis=1) == d_all).all()
    assert (np.concatenate([o1, o2], axis=1) == o_all).all()
    d_other, _ = sample(c, 3, 1, 0, N)        # other instance: other stream
    assert (d_other != d_all).any()


def test_pack_roundtrip():
    rng = np.random.default_rng(0)
    b = rng.random((5, 200)) < 0.5
    w = pack_bits(b)
    assert w.shape == (5, 4) and w.dtype == np.uint64
    assert (unpack_bits(w, 200) == b).all()
    assert int(w[0, 0]) & 1 == int(b[0, 0])
