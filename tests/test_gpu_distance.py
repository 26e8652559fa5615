"""The GPU circuit-distance search against the host search (Results, "Circuit-level
distance of distributed primitives"; Table I).

Both run the same breadth-first search over (active detection events, observable
mask) states; the GPU keeps the visited states in a fingerprint table and runs
whole levels at once.  With a state budget that suffices they return the same
weight.  The host search is pinned by brute force on the d = 3 memory DEM and by
Table I's surface-code rows (tests/test_library_host.py); the GPU search is
checked against it on surface-code and BB DEMs, exact (no cap on the active
set) where the DEM is small enough, capped elsewhere.
"""
import json
import os

import pytest

from workloads import MEMORY, NLCNOT, TELEPORT, bb, sc

pytestmark = pytest.mark.gpu

T1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))

CASES = [
    # (name, spec, max_active, max_weight)
    ("sc3-memory-exact", sc(3, MEMORY, 3, 0), 16, 8),
    ("sc3-nlcnot", sc(3, NLCNOT, 4, 3), 6, 10),
    ("sc3-teleport", sc(3, TELEPORT, 4, 3), 6, 10),
    ("sc5-nlcnot", sc(5, NLCNOT, 4, 3), 6, 12),
    ("bb18-nlcnot", bb("bb18", NLCNOT, 4, 3), 6, 12),
    ("bb36-memory", bb("bb36", MEMORY, 3, 0), 6, 12),
]


@pytest.mark.parametrize("name,spec,cap,wmax", CASES, ids=[c[0] for c in CASES])
def test_device_search_equals_host(gpu_lib, name, spec, cap, wmax):
    d = gpu_lib.DEM(gpu_lib.Circuit(spec))
    host = d.distance(max_active=cap, max_weight=wmax, max_states=20_000_000)
    dev = d.distance(max_active=cap, max_weight=wmax, max_states=20_000_000, device=True)
    print(f"[distance] {name}: host {host} device {dev}", flush=True)
    assert host > 0 and dev == host


@pytest.mark.parametrize("key", ["sc3", "sc5", "sc7"])
@pytest.mark.parametrize("op", [NLCNOT, TELEPORT])
def test_device_search_matches_table1(gpu_lib, key, op):
    d = gpu_lib.DEM(gpu_lib.Circuit(sc(int(key[2:]), op, 4, 3)))
    assert d.distance(max_active=6, max_weight=12, max_states=5_000_000, device=True) == T1[op][key]


def test_device_search_rejects_bad_arguments(gpu_lib):
    d = gpu_lib.DEM(gpu_lib.Circuit(sc(3, MEMORY, 3, 0)))
    with pytest.raises(gpu_lib.TmcsError):
        d.distance(max_active=17, device=True)
    with pytest.raises(gpu_lib.TmcsError):
        d.distance(max_states=0, device=True)
