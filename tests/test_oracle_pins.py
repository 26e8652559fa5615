"""Pins of the oracle's channel decomposition, symptom merging and exact ML decoding.

Each check compares the oracle with a fact fixed independently of its code:
  * the channel definitions of Methods "Simulation" (DEPOLARIZE1(p): X, Y, Z
    each with probability p/3; DEPOLARIZE2(p): each of the 15 non-identity
    two-qubit Paulis with probability p/15), enumerated exactly;
  * the XOR of two independent Bernoulli variables, enumerated exactly;
  * closed forms of maximum-likelihood decoding on repetition codes.
The last test plants plausible mistakes in the oracle (on the CPU) and checks
that these pins reject every one of them.
"""
import itertools
import math

import numpy as np
import pytest

import oracle.dem as odem
from oracle.bp import prior_llr
from oracle.circuits import Circuit
from oracle.ml import expected_ler, ml_ler

P_VALUES = [1e-4, 1e-3, 1e-2, 0.1, 0.3]

# symplectic bits of I, X, Y, Z
PX = (0, 1, 1, 0)
PZ = (0, 0, 1, 1)


def _mechanism_distribution(n_qubits, q):
    """Distribution over n-qubit Paulis (index = sum 4^k a_k) when each of the
    4^n - 1 non-identity Paulis is applied independently with probability q."""
    paulis = list(itertools.product(range(4), repeat=n_qubits))[1:]
    K = len(paulis)
    # symplectic vector of each mechanism as an integer (2 bits per qubit)
    vec = np.array([sum((PX[a] | PZ[a] << 1) << (2 * k) for k, a in enumerate(pl)) for pl in paulis],
                   dtype=np.int64)
    idx = np.arange(1 << K, dtype=np.int64)
    fires = (idx[:, None] >> np.arange(K)) & 1
    prob = np.prod(np.where(fires == 1, q, 1.0 - q), axis=1)
    acc = np.zeros(len(idx), dtype=np.int64)
    for k in range(K):
        acc ^= np.where(fires[:, k] == 1, vec[k], 0)
    out = np.zeros(4 ** n_qubits)
    np.add.at(out, acc, prob)
    return out


def _channel_distribution(n_qubits, p):
    """The depolarizing channel itself: identity 1 - p, every other Pauli p / (4^n - 1)
    (uniform over the non-identity Paulis, so any indexing that puts the identity
    at 0 - here the symplectic one of _mechanism_distribution - gives the same array)."""
    out = np.full(4 ** n_qubits, p / (4 ** n_qubits - 1))
    out[0] = 1.0 - p
    return out


def check_depolarize_mechanisms(component_prob=None):
    cp = component_prob or odem.component_prob
    for p in P_VALUES:
        for n, name in ((1, "DEPOLARIZE1"), (2, "DEPOLARIZE2")):
            got = _mechanism_distribution(n, cp(name, p))
            want = _channel_distribution(n, p)
            assert np.allclose(got, want, rtol=1e-9, atol=1e-15), (name, p)


def check_component_identities(component_prob=None):
    cp = component_prob or odem.component_prob
    for p in P_VALUES:
        q1 = cp("DEPOLARIZE1", p)
        q2 = cp("DEPOLARIZE2", p)
        # 1 - sqrt(1 - x) cancels: the rounding error is ~eps / x relative (< 1e-10 here)
        assert abs(q1 * (1 - q1) - p / 3) <= 1e-9 * p
        assert abs((1 - (1 - 2 * q2) ** 8) / 16 - p / 15) <= 1e-9 * p
        assert cp("X_ERROR", p) == p and cp("Z_ERROR", p) == p


def check_merge(merge=None):
    mp = merge or odem.merge_prob
    rng = np.random.default_rng(3)
    for pa, pb in list(itertools.product([0.0, 1e-3, 0.2, 0.5], repeat=2)) + \
            [tuple(rng.uniform(0, 0.5, 2)) for _ in range(20)]:
        odd = pa * (1 - pb) + pb * (1 - pa)          # enumeration of (a, b) with a xor b = 1
        assert abs(mp(pa, pb) - odd) <= 1e-15, (pa, pb)


def _circ(num_qubits, ops):
    c = Circuit()
    c.num_qubits = num_qubits
    for name, arg, t in ops:
        c.add(name, arg, t)
    return c


def _dem_joint(dem):
    """Exact joint distribution of the detector bits under the DEM's independent columns."""
    m = dem.num_dets
    out = np.zeros(1 << m)
    cols = dem.cols
    for fires in itertools.product([0, 1], repeat=len(cols)):
        pr = 1.0
        key = 0
        for f, (dets, _, p) in zip(fires, cols):
            pr *= p if f else 1 - p
            if f:
                for d in dets:
                    key ^= 1 << d
        out[key] += pr
    return out


def check_one_channel_dems():
    """DEMs of circuits with one or a few channels on freshly reset, then measured
    qubits: the joint detector distribution must equal the channels' own."""
    for p in (1e-3, 0.05, 0.3):
        # DEPOLARIZE1 before a Z (or X) measurement flips it with probability 2p/3
        for basis in ("Z", "X"):
            r, m = ("R", "M") if basis == "Z" else ("RX", "MX")
            c = _circ(1, [(r, None, [0]), ("DEPOLARIZE1", p, [0]), (m, None, [0]), ("DETECTOR", None, [0])])
            dem = odem.build_dem(c)
            assert len(dem.cols) == 1
            assert abs(dem.cols[0][2] - 2 * p / 3) <= 1e-14, (basis, p)
        # DEPOLARIZE2 on two qubits read out separately: (x0, x1) of the Pauli
        c = _circ(2, [("R", None, [0, 1]), ("DEPOLARIZE2", p, [0, 1]), ("M", None, [0, 1]),
                      ("DETECTOR", None, [0]), ("DETECTOR", None, [1])])
        dem = odem.build_dem(c)
        want = np.zeros(4)
        for a, b in itertools.product(range(4), repeat=2):      # Pauli a on qubit 0, b on qubit 1
            want[PX[a] | PX[b] << 1] += (1 - p) if a == b == 0 else p / 15
        assert len(dem.cols) == 3
        assert np.allclose(_dem_joint(dem), want, rtol=1e-12, atol=1e-15), p
        # a chain of channels on one qubit merges into one column
        p1, p2, p3 = p, 0.5 * p, 0.25 * p
        c = _circ(1, [("R", None, [0]), ("X_ERROR", p1, [0]), ("DEPOLARIZE1", p2, [0]),
                      ("Z_ERROR", 0.4, [0]), ("X_ERROR", p3, [0]), ("M", None, [0]), ("DETECTOR", None, [0])])
        dem = odem.build_dem(c)
        flip = 0.0
        for a, b, d in itertools.product([0, 1], repeat=3):    # X_ERROR, DEPOL flips the Z record, X_ERROR
            pr = (p1 if a else 1 - p1) * (2 * p2 / 3 if b else 1 - 2 * p2 / 3) * (p3 if d else 1 - p3)
            flip += pr * ((a + b + d) % 2)
        assert len(dem.cols) == 1
        assert abs(dem.cols[0][2] - flip) <= 1e-14, p


def test_depolarize_mechanisms_reproduce_channel():
    """The 3 (15) independent mechanisms give exactly the DEPOLARIZE1 (2) distribution."""
    check_depolarize_mechanisms()


def test_component_probability_identities():
    check_component_identities()


def test_merge_is_xor_of_bernoullis():
    check_merge()


def test_one_channel_dems_exact():
    check_one_channel_dems()


# ------------------------------------------------------------ exact ML / LER
def _repetition(n):
    H = np.zeros((n - 1, n), dtype=np.uint8)
    for i in range(n - 1):
        H[i, i] = H[i, i + 1] = 1
    L = np.zeros((1, n), dtype=np.uint8)
    L[0, 0] = 1
    return H, L


def check_ml_closed_forms(ml=None):
    """Repetition code of length n (odd) under i.i.d. flips p: ML fails exactly when
    more than half the bits flip, LER = sum_{k > n/2} C(n, k) p^k (1-p)^(n-k)."""
    fn = ml or ml_ler
    for n in (3, 5, 7):
        H, L = _repetition(n)
        for p in (0.01, 0.1, 0.3):
            want = sum(math.comb(n, k) * p ** k * (1 - p) ** (n - k) for k in range(n // 2 + 1, n + 1))
            got = fn(H, L, np.full(n, p))
            assert abs(got - want) <= 1e-12, (n, p, got, want)
    # n = 3 written out: p^3 + 3 p^2 (1 - p)
    H, L = _repetition(3)
    assert abs(fn(H, L, np.full(3, 0.2)) - (0.2 ** 3 + 3 * 0.04 * 0.8)) <= 1e-14


def test_ml_ler_closed_forms():
    check_ml_closed_forms()


def test_expected_ler_of_fixed_decoders():
    """A decoder that always predicts 'no flip' fails exactly when the observable
    flips: LER = P(bit 0 flips) = p_0; one that always predicts 'flip' fails with 1 - p_0."""
    H, L = _repetition(5)
    pri = np.array([0.07, 0.2, 0.01, 0.3, 0.15])
    zero = expected_ler(H, L, pri, lambda s: np.zeros((s.shape[0], 1), dtype=bool))
    one = expected_ler(H, L, pri, lambda s: np.ones((s.shape[0], 1), dtype=bool))
    assert abs(zero - 0.07) <= 1e-14 and abs(one - 0.93) <= 1e-14


def test_prior_llr_values():
    """lambda = ln((1-p)/p): 0 at p = 1/2, exactly k at p = 1/(1+e^k), odd about 1/2."""
    for k in (0.5, 1.0, 2.0, 6.0):
        p = 1.0 / (1.0 + math.exp(k))
        assert abs(prior_llr(np.array([p]))[0] - k) <= 1e-13 * max(1.0, k)
    assert prior_llr(np.array([0.5]))[0] == 0.0
    a = prior_llr(np.array([0.1, 0.9]))
    assert abs(a[0] + a[1]) <= 1e-15


# -------------------------------------------------- the pins catch mistakes
MUTANTS = {
    # DEPOLARIZE1 mechanisms at p/3 (first-order approximation)
    "q1=p/3": ("component_prob", lambda name, p: p / 3 if name == "DEPOLARIZE1" else _ORIG_CP(name, p)),
    # eighth root taken with two square roots (a fourth root)
    "q2 fourth root": ("component_prob", lambda name, p: (1 - math.sqrt(math.sqrt(1 - 16 * p / 15))) / 2
                       if name == "DEPOLARIZE2" else _ORIG_CP(name, p)),
    # q2 = p/15
    "q2=p/15": ("component_prob", lambda name, p: p / 15 if name == "DEPOLARIZE2" else _ORIG_CP(name, p)),
    # identical symptoms merged by adding probabilities
    "merge pa+pb": ("merge_prob", lambda pa, pb: pa + pb),
    # merge keeping the larger one
    "merge max": ("merge_prob", lambda pa, pb: max(pa, pb)),
}
_ORIG_CP = odem.component_prob


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistakes(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(odem, attr, fn)
    failed = 0
    for check in (check_depolarize_mechanisms, check_component_identities, check_merge, check_one_channel_dems):
        try:
            check()
        except AssertionError:
            failed += 1
    assert failed >= 1, name


@pytest.mark.parametrize("name", ["1 - sum P", "sum of min", "ML of flipped o"])
def test_ml_pin_rejects_planted_mistakes(name):
    from oracle.ml import enumerate_patterns, _key

    def wrong(H, L, pri):
        _, P, S, O = enumerate_patterns(H, L, pri)
        if name == "1 - sum P":
            return 1.0 - P.sum()
        best = {}
        for s, o, pr in zip(_key(S), _key(O), P):
            best.setdefault(int(s), {}).setdefault(int(o), 0.0)
            best[int(s)][int(o)] += pr
        if name == "sum of min":
            return 1.0 - sum(min(d.values()) for d in best.values())
        return 1.0 - sum(d.get(1, 0.0) for d in best.values())
    with pytest.raises(AssertionError):
        check_ml_closed_forms(wrong)
