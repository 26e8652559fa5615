"""Write the oracle's detector error models of large non-local CNOT circuits.

Building these with the oracle (single-fault injection in Python) takes minutes,
so the tests and the CPU-oracle leg of the benchmark load stored copies.  Only
oracle/ code runs here.  Each output dem_<name>.npz holds the columns as (column
pointer, sorted detector rows), the priors and the observable masks.

    python tests/golden/make_dems.py [name ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.circuits import build_circuit  # noqa: E402
from oracle.dem import build_dem  # noqa: E402
from workloads import NLCNOT, WORKLOADS, bb, pstring, sc  # noqa: E402

_MIX = WORKLOADS["sc_nlcnot_mixed"].specs
SPECS = {
    # the two d = 11 instances of the mixed batch (d/d rounds)
    "sc11_nlcnot_p1e-4": next(s for s in _MIX if s.d == 11 and s.p == 1e-4),
    "sc11_nlcnot_p1e-3": next(s for s in _MIX if s.d == 11 and s.p == 1e-3),
    # d = 21 and 29 at 3/3 rounds: the mixed batch's code sizes (frame beyond
    # 64 KB of LDS, BP state in device memory, windowed OSD) at a size the
    # oracle builds in minutes
    "sc21_nlcnot_r3_p1e-3": sc(21, NLCNOT, 3, 3, 1e-3, 1e-2),
    "sc29_nlcnot_r3_p1e-3": sc(29, NLCNOT, 3, 3, 1e-3, 1e-2),
    # Pauli-string compute of weight 5 (pattern 1010) on BB [[144,12,12]] blocks:
    # 6 blocks x 12 logicals = 72 observables (two mask words), one round first
    "bb144_pstring5_r1_p1e-3": pstring(bb("bb144", p=1e-3), 5, rounds=1),
}


def path(name):
    return os.path.join(HERE, "dem_%s.npz" % name)


def write(name):
    t0 = time.time()
    od = build_dem(build_circuit(SPECS[name]))
    col_ptr = [0]
    rows = []
    for dets, _, _ in od.cols:
        rows.extend(sorted(dets))
        col_ptr.append(len(rows))
    # observable masks: one uint64 per column, or [cols][words] beyond 64 observables
    ow = max(1, (od.num_obs + 63) // 64)
    obs = np.array([[(om >> (64 * w)) & ((1 << 64) - 1) for w in range(ow)] for _, om, _ in od.cols],
                   dtype=np.uint64)
    if ow == 1:
        obs = obs[:, 0]
    np.savez_compressed(path(name), num_dets=np.int64(od.num_dets), num_obs=np.int64(od.num_obs),
                        col_ptr=np.array(col_ptr, dtype=np.int32), rows=np.array(rows, dtype=np.int32),
                        priors=od.priors(), obs_mask=obs)
    print("wrote", path(name), od.num_dets, len(od.cols), "%.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or sorted(SPECS):
        write(n)
