"""GPU parity of the frame sampler: bit-exact against the oracle's frame propagator."""
import numpy as np
import pytest

from oracle.circuits import build_circuit
from oracle.frame import pack_bits, sample as oracle_sample
from workloads import MEMORY, NLCNOT, TELEPORT, WORKLOADS, bb, pstring, sc, with_decoherence

pytestmark = pytest.mark.gpu

CASES = [
    ("sc3-memory", sc(3, MEMORY, 3, 0, 1e-2)),
    ("sc3-nlcnot", sc(3, NLCNOT, 2, 2, 5e-3, 2e-2)),
    ("sc3-teleport", sc(3, TELEPORT, 2, 2, 5e-3, 2e-2)),
    ("bb18-teleport", bb("bb18", TELEPORT, 2, 2, 4e-3, 1e-2)),
    ("sc5-nlcnot", WORKLOADS["sc5_nlcnot"].specs[0]),
    ("bb144-memory", bb("bb144", MEMORY, 3, 0, 2e-3)),
    ("sc5-nlcnot-decoherence", with_decoherence(sc(5, NLCNOT, 3, 3, 1e-3, 1e-2), 0.01, False)),
    ("bb18-teleport-decoherence-lines", with_decoherence(bb("bb18", TELEPORT, 2, 2, 4e-3, 1e-2), 0.05, True)),
    ("sc5-pstring5", pstring(sc(5, p=2e-3), 5, rounds=2)),
    ("bb18-pstring4", pstring(bb("bb18", p=3e-3), 4, rounds=1)),
    # 17 blocks x 4 logicals = 68 observables: two observable words
    ("bb18-pstring16", pstring(bb("bb18", p=3e-3), 16, rounds=1)),
    # BB [[144,12,12]], weight 5 (pattern 1010): 72 observables
    ("bb144-pstring5", pstring(bb("bb144", p=1e-3), 5, rounds=1)),
]


def _lib_sample(tmcs, spec, seed, inst, begin, n):
    import torch
    c = tmcs.Circuit(spec)
    det, obs = c.alloc_outputs(n)
    det.fill_(-1)
    obs.fill_(-1)
    c.sample(seed, inst, begin, n, det, obs)
    torch.cuda.synchronize()
    return (det.cpu().numpy().view(np.uint64), obs.cpu().numpy().view(np.uint64)[: c.num_observables])


@pytest.mark.parametrize("name,spec", CASES, ids=[c[0] for c in CASES])
def test_sampler_bit_exact(gpu_lib, name, spec):
    oc = build_circuit(spec)
    for begin, n in ((0, 2 * 4096 + 100), (3 * 4096 + 5 * 64, 4096 + 37)):
        print(f"[sampler] {name} begin={begin} n={n}", flush=True)
        d_lib, o_lib = _lib_sample(gpu_lib, spec, 7, 2, begin, n)
        d_or, o_or = oracle_sample(oc, 7, 2, begin, n)
        assert (d_lib == pack_bits(d_or)).all()
        assert (o_lib == pack_bits(o_or)).all()


def test_sampler_full_size_subranges(gpu_lib):
    """The 10^6-shot run of the sc5 non-local CNOT workload agrees on sampled shot ranges."""
    import torch
    w = WORKLOADS["sc5_nlcnot"]
    spec = w.specs[0]
    c = gpu_lib.Circuit(spec)
    N = w.shots
    det, obs = c.alloc_outputs(N)
    c.sample(w.seed, 0, 0, N, det, obs)
    torch.cuda.synchronize()
    d = det.cpu().numpy().view(np.uint64)
    o = obs.cpu().numpy().view(np.uint64)
    oc = build_circuit(spec)
    for begin in (0, 123 * 4096 + 64 * 17, N - 4096 - 64 * 3):
        n = 4096 + 64 * 3 if begin + 4096 + 64 * 3 <= N else N - begin
        print(f"[sampler-full] begin={begin} n={n}", flush=True)
        d_or, o_or = oracle_sample(oc, w.seed, 0, begin, n)
        wb = begin // 64
        wn = (n + 63) // 64
        assert (d[:, wb:wb + wn] == pack_bits(d_or)).all()
        assert (o[:, wb:wb + wn] == pack_bits(o_or)).all()
    # the tail bits beyond N are zero
    if N % 64:
        assert (d[:, -1] >> np.uint64(N % 64) == 0).all()


def test_sampler_deterministic_and_composable(gpu_lib):
    spec = sc(3, NLCNOT, 2, 2, 5e-3, 2e-2)
    a, ao = _lib_sample(gpu_lib, spec, 11, 0, 0, 3 * 4096)
    b, bo = _lib_sample(gpu_lib, spec, 11, 0, 0, 3 * 4096)
    assert (a == b).all() and (ao == bo).all()
    p1, _ = _lib_sample(gpu_lib, spec, 11, 0, 0, 4096 + 64)
    p2, _ = _lib_sample(gpu_lib, spec, 11, 0, 4096 + 64, 2 * 4096 - 64)
    assert (np.concatenate([p1, p2], axis=1) == a).all()
    c, _ = _lib_sample(gpu_lib, spec, 11, 1, 0, 3 * 4096)
    assert (c != a).any()


def test_sampler_noiseless_is_zero(gpu_lib):
    d, o = _lib_sample(gpu_lib, bb("bb18", TELEPORT, 1, 1, 0.0, 0.0), 1, 0, 0, 5000)
    assert not d.any() and not o.any()


def test_sampler_rejects_bad_arguments(gpu_lib):
    import torch
    c = gpu_lib.Circuit(sc(3, MEMORY, 3, 0))
    det, obs = c.alloc_outputs(128)
    with pytest.raises(gpu_lib.TmcsError):
        c.sample(1, 0, 32, 64, det, obs)   # shot_begin not a multiple of 64
    torch.cuda.synchronize()


def test_async_sample_and_error_count_match_the_waiting_calls(gpu_lib):
    """tmcs_sample_async writes the same bits as tmcs_sample (two shot ranges,
    the second at an offset and ragged) and leaves the overflow flag clear;
    tmcs_count_errors accumulates the count tmcs_logical_error_rate returns."""
    import torch
    spec = sc(5, NLCNOT, 5, 5, 3e-3, 2e-2)
    print("[sampler] async sc5-nlcnot", flush=True)
    c = gpu_lib.Circuit(spec)
    dem = gpu_lib.DEM(c)
    k = c.num_observables
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    for begin, n in ((0, 3 * 4096), (64 * 1000, 4096 + 70)):
        det, obs = c.alloc_outputs(n)
        c.sample(7, 0, begin, n, det, obs)
        det2, obs2 = c.alloc_outputs(n)
        c.sample_async(7, 0, begin, n, det2, obs2, flag)
        torch.cuda.synchronize()
        assert torch.equal(det, det2) and torch.equal(obs, obs2), begin
        assert int(flag.item()) == 0
        pred = torch.zeros_like(obs)
        dem.decode(det, n, pred, max_iter=30)
        ne, _, _ = gpu_lib.logical_error_rate(pred, obs, k, n)
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        gpu_lib.count_errors(pred, obs, k, n, cnt)
        gpu_lib.count_errors(pred, obs, k, n, cnt)
        torch.cuda.synchronize()
        assert ne > 0 and int(cnt.item()) == 2 * ne, (begin, ne, int(cnt.item()))
