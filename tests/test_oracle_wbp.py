"""Pin the weighted-BP oracle gradient with central finite differences."""
import numpy as np
import pytest

from oracle.bp import decode_bp
from oracle.codes import surface_code
from oracle.wbp import backward, forward


def _problem(seed, T):
    rng = np.random.default_rng(seed)
    c = surface_code(3)
    H = np.vstack([c.hz, c.hx])               # 8 x 9, checks of degree 2 and 4
    n = H.shape[1]
    priors = rng.uniform(0.02, 0.2, size=n)
    e = rng.random((3, n)) < 0.25
    synd = (e.astype(int) @ H.T) % 2 == 1
    E = int(H.sum())
    W = rng.uniform(0.6, 1.4, size=(T, E))
    G = rng.normal(size=(T, 3, n))
    return H, priors, synd, W, G


@pytest.mark.parametrize("seed", range(4))
def test_gradient_matches_central_differences(seed):
    T = 4
    H, priors, synd, W, G = _problem(seed, T)
    f = forward(H, priors, synd, W)
    gW = backward(f, G)
    loss = lambda Wx: float(np.sum(G * forward(H, priors, synd, Wx)["L"]))
    h = 1e-6
    rng = np.random.default_rng(100 + seed)
    idx = [(int(rng.integers(T)), int(rng.integers(W.shape[1]))) for _ in range(25)]
    for t, e in idx:
        Wp, Wm = W.copy(), W.copy()
        Wp[t, e] += h
        Wm[t, e] -= h
        fd = (loss(Wp) - loss(Wm)) / (2 * h)
        assert abs(fd - gW[t, e]) <= 1e-5 * max(1.0, abs(fd)), (t, e, fd, gW[t, e])


def test_forward_with_unit_weights_is_plain_min_sum():
    T = 5
    H, priors, synd, W, _ = _problem(7, T)
    f = forward(H, priors, synd, np.ones_like(W))
    r = decode_bp(H, priors, synd, T, early_stop=False)
    assert np.allclose(f["L"][-1], r["llr"], rtol=0, atol=1e-12)
    r2 = decode_bp(H, priors, synd, 2, early_stop=False)
    assert np.allclose(f["L"][1], r2["llr"], rtol=0, atol=1e-12)


def test_forward_fp32_matches_weighted_decoder_fp32():
    T = 6
    H, priors, synd, W, _ = _problem(3, T)
    f = forward(H, priors, synd, W, dtype=np.float32)
    r = decode_bp(H, priors, synd, T, weights=W.astype(np.float32), dtype=np.float32, early_stop=False)
    assert (f["L"][-1] == r["llr"]).all()
