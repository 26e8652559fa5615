"""CPU tests of the C ABI's argument checks: calls that must fail (or return
early) before any device work, so they run without a GPU."""
import ctypes
import os

import pytest

from workloads import MEMORY, sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OK, EINVAL = 0, 1


@pytest.fixture(scope="module")
def lib():
    so = os.path.join(ROOT, "paper_2504_05611_amd", "libtmcs.so")
    if not os.path.exists(so):
        from paper_2504_05611_amd.build import build
        build(verbose=False)
    from paper_2504_05611_amd import tmcs
    return tmcs


@pytest.fixture(scope="module")
def handles(lib):
    c = lib.Circuit(sc(3, MEMORY, 3, 0))
    return c, lib.DEM(c)


def _err(lib):
    return lib._lib.tmcs_last_error().decode()


def test_decoder_config_is_validated(lib, handles):
    _, d = handles
    raw = lib._lib
    cfg = lib.make_cfg(max_iter=0)
    assert raw.tmcs_decode(d._h, ctypes.byref(cfg), None, 64, None, None, None) == EINVAL
    assert "max_iter" in _err(lib)
    cfg = lib.make_cfg(max_iter=10, alpha=0.0)
    assert raw.tmcs_decode(d._h, ctypes.byref(cfg), None, 64, None, None, None) == EINVAL
    assert "alpha" in _err(lib)
    for w in (-1, 2049):
        cfg = lib.make_cfg(max_iter=10, osd_window=w)
        assert raw.tmcs_decode(d._h, ctypes.byref(cfg), None, 64, None, None, None) == EINVAL
        assert "osd_window" in _err(lib)
    for o in (-1, 65):
        cfg = lib.make_cfg(max_iter=10, osd_order=o)
        assert raw.tmcs_decode(d._h, ctypes.byref(cfg), None, 64, None, None, None) == EINVAL
        assert "osd_order" in _err(lib)
    for ch in (-64, 100):
        cfg = lib.make_cfg(max_iter=10, decode_chunk=ch)
        assert raw.tmcs_decode(d._h, ctypes.byref(cfg), None, 64, None, None, None) == EINVAL
        assert "decode_chunk" in _err(lib)
    cfg = lib.make_cfg(max_iter=10)
    assert raw.tmcs_decode(None, ctypes.byref(cfg), None, 64, None, None, None) == EINVAL
    # no shots: nothing to do, no device work
    assert raw.tmcs_decode(d._h, ctypes.byref(cfg), None, 0, None, None, None) == OK


def test_sample_arguments_are_validated(lib, handles):
    c, _ = handles
    raw = lib._lib
    assert raw.tmcs_sample(c._h, 1, 0, 32, 64, None, None, None) == EINVAL     # shot_begin % 64
    assert "multiple of 64" in _err(lib)
    assert raw.tmcs_sample(c._h, 1, 0, 0, 0, None, None, None) == OK           # empty range
    assert raw.tmcs_sample(None, 1, 0, 0, 64, None, None, None) == EINVAL
    # the non-waiting variants need their device flag / counter
    assert raw.tmcs_sample_async(c._h, 1, 0, 0, 64, None, None, None, None) == EINVAL
    assert "overflow" in _err(lib)
    assert raw.tmcs_count_errors(None, None, 1, 64, None, None) == EINVAL
    assert "counter" in _err(lib)


def test_plan_arguments_are_validated(lib, handles):
    c, d = handles
    raw = lib._lib
    out = ctypes.c_void_p()
    items = (lib.PlanItem * 1)()
    items[0].circuit, items[0].dem = c._h, d._h
    items[0].cfg = lib.make_cfg(max_iter=10)
    assert raw.tmcs_plan_create(items, 1, 1000, 1, ctypes.byref(out)) == EINVAL    # not a multiple of 4096
    assert "4096" in _err(lib)
    assert raw.tmcs_plan_create(None, 1, 4096, 1, ctypes.byref(out)) == EINVAL
    assert raw.tmcs_plan_create(items, 0, 4096, 1, ctypes.byref(out)) == EINVAL
    items[0].cfg.iters_dev = 16     # any non-null pointer: refused before it is used
    assert raw.tmcs_plan_create(items, 1, 4096, 1, ctypes.byref(out)) == EINVAL    # per-shot outputs
    assert not out.value


def test_weighted_bp_workspace_size(lib, handles):
    _, d = handles
    raw = lib._lib
    n = ctypes.c_size_t()
    assert raw.tmcs_wbp_workspace_size(d._h, 4, 100, ctypes.byref(n)) == OK
    small, large = ctypes.c_size_t(), ctypes.c_size_t()
    raw.tmcs_wbp_workspace_size(d._h, 4, 100, ctypes.byref(small))
    raw.tmcs_wbp_workspace_size(d._h, 8, 200, ctypes.byref(large))
    assert large.value >= 4 * small.value - 4096     # linear in T x shots (up to alignment)
    assert raw.tmcs_wbp_workspace_size(d._h, 0, 100, ctypes.byref(n)) == EINVAL
