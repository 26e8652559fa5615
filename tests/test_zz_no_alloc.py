"""The no-allocation sampler (tmcs_sample_noalloc) against tmcs_sample_async.

tmcs_sample_noalloc draws the same shots as tmcs_sample_async but keeps its
event scratch in the library's fixed device array instead of buffers it
allocates.  Both are called through the raw C ABI on the same shot ranges,
twice in a row with the second call smaller, and their outputs must be
identical bit for bit.
"""
import numpy as np
import pytest

from workloads import MEMORY, NLCNOT, WORKLOADS, bb, sc

pytestmark = pytest.mark.gpu


def _noalloc(t, circ, seed, inst, begin, n, det, obs, flag):
    """The raw C entry point (ctypes argument types as declared in tmcs.h)."""
    st = t._lib.tmcs_sample_noalloc(circ._h, seed, inst, begin, n, t._ptr(det), t._ptr(obs), t._ptr(flag),
                                    t._stream(None))
    if st != 0:
        raise t.TmcsError(st, t._lib.tmcs_last_error().decode())


def _async(circ, seed, inst, begin, n, flag):
    det, obs = circ.alloc_outputs(n)
    circ.sample_async(seed, inst, begin, n, det, obs, flag)
    return det, obs


# (spec, calls (shot_begin, n_shots)): the second call of each case is smaller;
# BB144 memory needs ~1.6 MB of scratch per 4096-shot block, so its 2^18-shot
# call runs in several chunks of the 64 MiB scratch where the growing path uses one
CASES = {
    "sc5_nlcnot": (WORKLOADS["sc5_nlcnot"].specs[0], [(64 * 7, 3 * 4096 + 200), (4096 * 5, 1000)]),
    "sc3_memory": (sc(3, MEMORY, 3, 0, 2e-2), [(0, 9000), (128, 77)]),
    "bb144_memory": (bb("bb144", MEMORY, 12, 0, 2e-3), [(0, 1 << 18), (4096 * 3, 4096 + 64)]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_noalloc_sampler_equals_async(gpu_lib, name):
    import torch
    t = gpu_lib
    spec, calls = CASES[name]
    circ = t.Circuit(spec)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    circ.sample_async(1, 0, 0, 64, *circ.alloc_outputs(64), flag)     # puts the program on the device
    for begin, n in calls:
        det_ref, obs_ref = _async(circ, 7, 2, begin, n, flag)
        det, obs = circ.alloc_outputs(n)
        det.fill_(-1)
        obs.fill_(-1)
        _noalloc(t, circ, 7, 2, begin, n, det, obs, flag)
        torch.cuda.synchronize()
        assert int(flag.item()) == 0
        assert torch.equal(det, det_ref), (name, begin, n)
        assert torch.equal(obs, obs_ref), (name, begin, n)


def test_noalloc_sampler_rejects_what_it_cannot_do(gpu_lib):
    """Host-side errors: a circuit whose program is not on the device yet, a
    missing overflow flag, and a circuit whose event scratch for one 4096-shot
    block exceeds the fixed array (d = 7 non-local CNOT, 4/4 rounds, p = 0.45:
    ~2.5 k events per shot, ~100 MB per block)."""
    import torch
    t = gpu_lib
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    fresh = t.Circuit(sc(3, MEMORY, 3, 0))
    det, obs = fresh.alloc_outputs(64)
    with pytest.raises(t.TmcsError) as e:
        _noalloc(t, fresh, 1, 0, 0, 64, det, obs, flag)
    assert e.value.status == 1 and "not on this device" in str(e.value)
    fresh.sample_async(1, 0, 0, 64, det, obs, flag)
    with pytest.raises(t.TmcsError) as e:
        _noalloc(t, fresh, 1, 0, 0, 64, det, obs, None)
    assert e.value.status == 1
    heavy = t.Circuit(sc(7, NLCNOT, 4, 4, 0.45, 0.45))
    d2, o2 = heavy.alloc_outputs(64)
    heavy.sample_async(1, 0, 0, 64, d2, o2, flag)
    with pytest.raises(t.TmcsError) as e:
        _noalloc(t, heavy, 1, 0, 0, 64, d2, o2, flag)
    assert e.value.status == 4 and "no-allocation scratch holds" in str(e.value)
    torch.cuda.synchronize()
