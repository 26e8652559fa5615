"""CPU tests of the library's host side: ABI symbols, circuits and DEMs vs the oracle.

These call only host-side entry points (circuit and DEM construction); nothing
here touches a GPU.
"""
import os
import re

import numpy as np
import pytest

from oracle.circuits import build_circuit
from oracle.dem import build_dem
from workloads import MEMORY, NLCNOT, TELEPORT, WORKLOADS, bb, pstring, sc, with_decoherence

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    so = os.path.join(ROOT, "paper_2504_05611_amd", "libtmcs.so")
    if not os.path.exists(so):
        from paper_2504_05611_amd.build import build
        build(verbose=False)
    from paper_2504_05611_amd import tmcs
    return tmcs


def test_exports_every_declared_symbol(lib):
    text = open(os.path.join(ROOT, "include", "tmcs.h")).read()
    declared = set(re.findall(r"\b(tmcs_[a-z0-9_]+)\s*\(", text))
    assert len(declared) >= 15
    import ctypes
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(so, name), name
    assert declared == set(lib.EXPORTED)


SPECS = [sc(3, MEMORY, 3, 0), sc(3, NLCNOT, 4, 3, 1e-3, 1e-2), sc(3, TELEPORT, 4, 3),
         sc(5, NLCNOT, 5, 5, 1e-3, 1e-2), bb("bb18", NLCNOT, 4, 3), bb("bb18", TELEPORT, 4, 3),
         bb("bb36", MEMORY, 2, 0, 2e-3),
         with_decoherence(sc(3, NLCNOT, 4, 3, 1e-3, 1e-2), 0.05, False),
         with_decoherence(sc(5, NLCNOT, 3, 3, 1e-3, 1e-3), 0.02, True),
         with_decoherence(bb("bb18", TELEPORT, 4, 3), 0.01, True),
         pstring(sc(3), 2), pstring(sc(5), 5), pstring(bb("bb18"), 4, rounds=2)]


@pytest.mark.parametrize("spec", SPECS, ids=lambda s: f"{s.code}{s.d if s.code == 'sc' else s.bb}-{s.op}"
                         + (f"-decoh{s.ebit_per_step}" if s.ebit_per_step else "")
                         + (f"{s.weight}" if s.op == "pstring" else ""))
def test_circuit_and_dem_match_oracle(lib, spec):
    lc = lib.Circuit(spec)
    oc = build_circuit(spec)
    assert lc.text() == oc.text()
    k = oc.counts()
    assert lc.info["detectors"] == k["dets"] and lc.info["noise_sites"] == k["sites"]
    assert lc.info["gates_1q"] == k["q1"] and lc.info["gates_2q"] == k["q2"]
    # expected noise events per shot: one Bernoulli(p) event per site of every noise instruction
    ev = sum(arg * (len(t) // 2 if name == "DEPOLARIZE2" else len(t))
             for name, arg, t in oc.ops if name in ("X_ERROR", "Z_ERROR", "DEPOLARIZE1", "DEPOLARIZE2"))
    assert lc.info["events_per_mshot"] == round(ev * 1e6)
    ld = lib.DEM(lc)
    od = build_dem(oc)
    assert ld.cols == od.num_cols and ld.rows == od.num_dets
    h = ld.export()
    assert (ld.H() == od.H()).all()
    assert (h.priors == od.priors()).all()                      # same FP64 operations, same order
    assert (h.obs_mask == np.array([c[1] for c in od.cols], dtype=np.uint64)).all()
    from oracle.codes import rank
    assert ld.info["rank"] == rank(od.H())


@pytest.mark.slow
@pytest.mark.parametrize("name", ["bb144_memory", "bb144_teleport"])
def test_full_size_dem_matches_oracle(lib, name):
    spec = WORKLOADS[name].specs[0]
    lc = lib.Circuit(spec)
    oc = build_circuit(spec)
    assert lc.text() == oc.text()
    ld = lib.DEM(lc)
    od = build_dem(oc)
    assert (ld.H() == od.H()).all() and (ld.export().priors == od.priors()).all()


def test_invalid_specs_are_rejected(lib):
    with pytest.raises(lib.TmcsError):
        lib.Circuit(sc(4, MEMORY, 3, 0))                       # even distance
    with pytest.raises(lib.TmcsError):
        lib.Circuit(sc(3, NLCNOT, 3, 0))                       # no rounds after the CNOT
    with pytest.raises(lib.TmcsError):
        lib.Circuit(sc(3, MEMORY, 3, 0, p=0.7))


def test_distance_search_is_exact_on_a_small_dem(lib):
    """With no cap on the active detection events the search returns the minimum
    weight of an undetectable logical error: brute force over all sets of up to
    three mechanisms of the d = 3 memory DEM (55 columns)."""
    import itertools
    d = lib.DEM(lib.Circuit(sc(3, MEMORY, 3, 0)))
    H = d.H().astype(np.int64)
    om = d.export().obs_mask
    best = None
    for w in (1, 2, 3):
        for cs in itertools.combinations(range(d.cols), w):
            if not (H[:, list(cs)].sum(axis=1) % 2).any() and np.bitwise_xor.reduce(om[list(cs)]):
                best = w
                break
        if best:
            break
    assert best == 3
    assert d.distance(max_active=d.rows, max_weight=6) == best


@pytest.mark.parametrize("op", ["nlcnot", "teleport"])
@pytest.mark.parametrize("key", ["sc3", "sc5", "sc7"])
def test_distance_search_matches_table1(lib, key, op):
    import json
    t1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    spec = sc(int(key[2:]), NLCNOT if op == "nlcnot" else TELEPORT, 4, 3)
    d = lib.DEM(lib.Circuit(spec))
    assert d.distance(max_active=6, max_weight=12, max_states=5_000_000) == t1[op][key]


def test_nondeterministic_outputs_are_rejected(tmp_path):
    """The DEM builder's noiseless-determinism check (ENONDETERMINISTIC = 5) on
    hand-written circuits whose answer is textbook stabilizer algebra: a |+>
    measured in Z, H on a fresh qubit, one half of a Bell pair and an
    uncorrected teleportation are random; repeated measurements, the ZZ and XX
    parities of a Bell pair and a corrected teleportation are deterministic."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    csrc = os.path.join(ROOT, "paper_2504_05611_amd", "csrc")
    exe = str(tmp_path / "nondet_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
                    os.path.join(ROOT, "tests", "native", "nondet_check.cpp"),
                    os.path.join(csrc, "host", "dem.cpp"), os.path.join(csrc, "host", "codes.cpp"),
                    "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.splitlines()
    got = {line.split()[0]: (int(line.split()[1]), " ".join(line.split()[2:])) for line in out}
    det = ["reset_measure", "repeat_measure", "bell_zz", "bell_xx", "teleport_corrected"]
    rand = ["rx_measure_z", "start_h_measure", "bell_half", "bell_zx", "teleport_uncorrected", "random_observable"]
    for name in det:
        assert got[name][0] == 0, (name, got[name])
    for name in rand:
        assert got[name][0] == 5, (name, got[name])
    assert got["random_observable"][1].startswith("observable 0")
    assert got["bell_half"][1].startswith("detector 0")


def test_host_builders_under_sanitizers(tmp_path):
    """The circuit, code, DEM, program and distance builders, built with g++ under
    AddressSanitizer and UndefinedBehaviorSanitizer (any report aborts the run),
    on surface-code and BB memory, non-local CNOT, teleportation, decoherence and
    Pauli-string circuits; invalid specs fail with TMCS_EINVAL.  The exact
    distance searches give the code distance 3 of the d = 3 operations (Table I)
    and 3 for the [[18,4,4]] memory circuit."""
    import shutil
    import subprocess
    from concurrent.futures import ThreadPoolExecutor
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    csrc = os.path.join(ROOT, "paper_2504_05611_amd", "csrc")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-I" + os.path.join(ROOT, "include"), "-I" + csrc]
    srcs = [os.path.join(ROOT, "tests", "native", "host_sanitize.cpp")] + [
        os.path.join(csrc, "host", f + ".cpp") for f in ("circuit", "codes", "dem", "distance", "program")]
    objs = [str(tmp_path / (os.path.basename(x) + ".o")) for x in srcs]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        for r in ex.map(lambda so: subprocess.run([gxx] + flags + ["-c", so[0], "-o", so[1]], capture_output=True,
                                                  text=True), zip(srcs, objs)):
            assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "host_sanitize")
    subprocess.run([gxx, "-fsanitize=address,undefined"] + objs + ["-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    got = {line.split()[0]: [int(x) for x in line.split()[1:]] for line in r.stdout.splitlines()}
    assert len(got) == 15
    for name, (st, dets, cols, edges, dist) in got.items():
        if name.startswith("bad_"):
            assert st == 1, name
        else:
            assert st == 0 and dets > 0 and cols > 0 and edges >= cols, (name, st)
    for name in ("sc3_memory", "sc3_nlcnot", "sc3_teleport", "bb18_memory"):
        assert got[name][4] == 3, (name, got[name])


def test_more_than_64_observables_match_oracle(lib):
    """A Pauli string of weight 16 on [[18,4,4]] blocks has 17 x 4 = 68 observables:
    the DEM's masks take two words per column, and columns with equal detector
    lists are ordered by the mask read as one integer (the oracle's Python int)."""
    spec = pstring(bb("bb18", p=4e-3), 16, rounds=1)
    lc = lib.Circuit(spec)
    oc = build_circuit(spec)
    assert lc.text() == oc.text()
    ld = lib.DEM(lc)
    od = build_dem(oc)
    assert ld.info["obs"] == od.num_obs == 68
    h = ld.export()
    assert h.obs_mask.shape == (od.num_cols, 2)
    want = np.array([[(om >> (64 * w)) & ((1 << 64) - 1) for w in range(2)] for _, om, _ in od.cols],
                    dtype=np.uint64)
    assert (h.obs_mask == want).all()
    assert (ld.H() == od.H()).all() and (h.priors == od.priors()).all()
    assert (ld.L() == od.L()).all()
    with pytest.raises(lib.TmcsError):
        ld.distance()                                       # the search keeps one mask word


@pytest.mark.slow
def test_bb_schedule_keeps_the_code_distance(lib):
    """The interleaved BB cycle (R16) keeps the circuit distance of the [[36,4,6]]
    memory circuit at the code distance 6 (Table IV); the capped search finds a
    weight-6 logical error and none lighter within its cap.  The earlier
    Z-checks-then-X-checks order dropped it to 4."""
    d = lib.DEM(lib.Circuit(bb("bb36", MEMORY, 3, 0)))
    assert d.distance(max_active=6, max_weight=12, max_states=20_000_000) == 6
