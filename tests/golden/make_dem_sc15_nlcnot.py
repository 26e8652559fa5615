"""Write the oracle's detector error model of the d=15 non-local CNOT workload.

Building it with the oracle (single-fault injection in Python) takes minutes,
so the parity test of the device-memory BP path loads this stored copy.  Only
oracle/ code runs here.  Output: dem_sc15_nlcnot_p1e-3.npz with the columns as
(column pointer, sorted detector rows), the priors, and the observable masks.

    python tests/golden/make_dem_sc15_nlcnot.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.circuits import build_circuit  # noqa: E402
from oracle.dem import build_dem  # noqa: E402
from workloads import WORKLOADS  # noqa: E402

SPEC = next(s for s in WORKLOADS["sc_nlcnot_mixed"].specs if s.d == 15 and s.p == 1e-3)
PATH = os.path.join(HERE, "dem_sc15_nlcnot_p1e-3.npz")


def main():
    od = build_dem(build_circuit(SPEC))
    col_ptr = [0]
    rows = []
    for dets, _, _ in od.cols:
        rows.extend(sorted(dets))
        col_ptr.append(len(rows))
    obs = np.array([om for _, om, _ in od.cols], dtype=np.uint64)
    np.savez_compressed(PATH, num_dets=np.int64(od.num_dets), num_obs=np.int64(od.num_obs),
                        col_ptr=np.array(col_ptr, dtype=np.int32), rows=np.array(rows, dtype=np.int32),
                        priors=od.priors(), obs_mask=obs)
    print("wrote", PATH, od.num_dets, len(od.cols))


if __name__ == "__main__":
    main()
