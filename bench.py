"""Benchmark: shots/s of the whole shot pipeline (sample + BP-OSD decode + LER) on one GPU.

One step = one pass of the hot path over one batch of synthetic shots of the
workload: Pauli-frame sampling of the batch (a new shot range every step),
BP + OSD-0 decoding of every syndrome, and the logical-error count.  The
circuit and its detector error model are built once, before timing.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
Prints ONE JSON line.  Multi-GPU runs are not part of this build.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# plain 32-bit VALU lane operations: 256 CUs x 64 lanes per clock x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
BP_OPS_PER_EDGE_ITER = 10      # |q|, two min compares, sign XORs, message rebuild, add
FRAME_OPS_PER_CX_WORD = 4      # two 64-bit XORs per CX per 64-shot word
# whole-sampler model (frame bit-ops plus the prescribed random numbers): a
# Philox4x32-10 call is ~220 issue slots (quarter-rate 32-bit multiplies) for 4
# draws, one draw starts every (site, 4096-shot block) stream, and an event costs
# a gap draw, a component draw, a 12-step table search and its frame update
PHILOX_OPS_PER_DRAW = 55
GAP_SEARCH_OPS = 36
EVENT_APPLY_OPS = 4

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch,
# averaged over the dispatches of a --steps 1 --warmup 1 run of this workload),
# scaled by what the counters read for a plain 1 GiB device copy.  Valid only for
# the sources they were taken on: the SHA-256 of those files, in order, must match.
# Commands and raw figures: profiles/hbm_traffic_sc5_nlcnot.md
TRAFFIC = {
    "sc5_nlcnot": {
        "k_bp": {"src": ['paper_2504_05611_amd/csrc/kernels/decode.hip'],
                 "sha256": "03be1640d29e262e7fa79b55d7c89ae35d2a88b8fc854330c6b0d2413b9f1bfa",
                 "fetch_kib": 72915.6, "write_kib": 133335.7},
        "k_frame": {"src": ['paper_2504_05611_amd/csrc/kernels/sample.hip', 'paper_2504_05611_amd/csrc/host/program.cpp'],
                    "sha256": "a995ee3c19865f8598c874400fecec85e360bbb766f1e7164d0f5f422eff8eb4",
                    "fetch_kib": 59909.7, "write_kib": 38549.7},
    },
}
FETCH_SCALE = 1048576.0 / 524302.5   # copy-kernel calibration (1 GiB read per launch)
WRITE_SCALE = 1048576.0 / 1048576.0


def traffic_bytes(workload, kernel):
    """Scaled HBM bytes per launch, or None when no counters match the current source."""
    import hashlib
    t = TRAFFIC.get(workload, {}).get(kernel)
    if t is None:
        return None
    h = hashlib.sha256()
    for src in t["src"]:                      # every source the counted kernel depends on
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != t["sha256"]:
        return None
    return (t["fetch_kib"] * FETCH_SCALE + t["write_kib"] * WRITE_SCALE) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sc5_nlcnot")
    ap.add_argument("--shots", type=int, default=0, help="override the workload's batch size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 1 << 27                      # 2^27 int64 = 1 GiB
    a = torch.ones(n, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 8, "launches": 3}))


def _cpu_worker(spec, seed, begin, n, bp_iters, barrier, q):
    """One host process of the all-cores leg: oracle sample + BP-OSD decode of shots [begin, begin + n)."""
    from threadpoolctl import threadpool_limits

    from oracle.circuits import build_circuit
    from oracle.dem import build_dem
    from oracle.frame import sample
    from oracle.osd import Decoder
    with threadpool_limits(limits=1):
        oc = build_circuit(spec)
        od = build_dem(oc)
        dec = Decoder(od.H(), od.priors(), od.L(), max_iter=bp_iters, dtype=__import__("numpy").float64)
        barrier.wait()
        t0 = time.perf_counter()
        det, _ = sample(oc, seed, 0, begin, n)
        dec.decode(det.T)
        q.put((t0, time.perf_counter()))


def cpu_baseline_all_cores(w, spec, per_proc=1024):
    """The oracle in one process per host core (at most 16), each on its own slice of the
    workload's shots: total shots / (last finish - first start)."""
    import multiprocessing as mp
    nproc = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    barrier, q = ctx.Barrier(nproc), ctx.Queue()
    procs = [ctx.Process(target=_cpu_worker, args=(spec, w.seed, i * per_proc, per_proc, w.bp_iters, barrier, q))
             for i in range(nproc)]
    for p in procs:
        p.start()
    times = [q.get(timeout=600) for _ in procs]
    for p in procs:
        p.join()
    wall = max(t[1] for t in times) - min(t[0] for t in times)
    return dict(value=nproc * per_proc / wall, unit="shots/s", cores=nproc, kind="oracle",
                sample=f"{nproc} processes x {per_proc} shots (shots [0, {nproc * per_proc}), seed {w.seed}), "
                       f"one host thread each; FP64 oracle sample + BP-OSD decode, {wall:.2f} s wall")


def cpu_baseline(w, spec, n_shots):
    """Time the oracle (as it stands) on a bounded sample of the workload on host cores."""
    from threadpoolctl import threadpool_limits

    from oracle.circuits import build_circuit
    from oracle.dem import build_dem
    from oracle.frame import sample
    from oracle.osd import Decoder
    with threadpool_limits(limits=1):
        oc = build_circuit(spec)
        od = build_dem(oc)
        dec = Decoder(od.H(), od.priors(), od.L(), max_iter=w.bp_iters, dtype=__import__("numpy").float64)
        t0 = time.perf_counter()
        det, obs = sample(oc, w.seed, 0, 0, n_shots)
        t1 = time.perf_counter()
        dec.decode(det.T)
        t2 = time.perf_counter()
    return dict(value=n_shots / (t2 - t0), unit="shots/s", cores=1, kind="oracle",
                sample=f"{n_shots} shots of the same workload (shots [0, {n_shots}), seed {w.seed}); "
                       f"FP64 oracle: frame sampling {t1 - t0:.2f} s + BP-OSD decode {t2 - t1:.2f} s, "
                       f"one host thread")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: only one GPU is used in this build (asked for --gpus {args.gpus}); "
              "the path would shard by 4096-shot noise blocks with one all-reduce of the counts.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration()
        return
    from paper_2504_05611_amd import tmcs
    from workloads import WORKLOADS

    w = WORKLOADS[args.workload]
    spec = w.specs[0]
    shots = args.shots or w.shots
    # host baselines first, before this process initialises the GPU (the all-cores
    # leg starts fresh interpreter processes)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_all_cores(w, spec)
        cpu["single_thread"] = cpu_baseline(w, spec, 8192)
    torch.cuda.set_device(0)
    circ = tmcs.Circuit(spec)
    dem = tmcs.DEM(circ)
    det, obs = circ.alloc_outputs(shots)
    pred = torch.zeros_like(obs)
    stats = tmcs.new_stats()
    k = circ.num_observables

    # a step never waits: the sampler's event-buffer overflow flag and the
    # failing-shot count stay on the device and are read after the timed steps
    overflow = torch.zeros(1, dtype=torch.int32, device="cuda")
    n_err = torch.zeros(1, dtype=torch.int64, device="cuda")

    def step(i):
        circ.sample_async(w.seed, 0, i * shots, shots, det, obs, overflow)
        dem.decode(det, shots, pred, max_iter=w.bp_iters, stats=stats)
        tmcs.count_errors(pred, obs, k, shots, n_err)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    stats.zero_()
    n_err.zero_()
    tmcs.timing_reset()
    tmcs.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if int(overflow.item()):
        raise RuntimeError("noise event buffer overflow during the timed steps")
    errors = int(n_err.item())
    tmcs.timing_enable(False)
    kern = tmcs.timing_report()
    st = tmcs.read_stats(stats)
    elapsed = t1 - t0
    total = shots * args.steps
    value = total / elapsed

    sample_ms = sum(v[1] for n, v in kern.items() if n.startswith(("k_event", "k_scan", "k_frame", "k_zero_u32")))
    decode_ms = sum(v[1] for n, v in kern.items()
                    if n in ("k_bp", "k_osd", "k_osd_retry", "k_compact", "k_zero_i32", "k_add_shots"))
    dominant = max(kern.items(), key=lambda kv: kv[1][1])[0]
    launches, dom_ms = kern[dominant]
    avg_s = dom_ms / launches / 1e3
    info = circ.info
    if dominant == "k_bp":
        ops = BP_OPS_PER_EDGE_ITER * dem.edges * st["bp_iters"] / launches
        model = (f"{BP_OPS_PER_EDGE_ITER} lane-ops per edge per BP iteration x {dem.edges} edges x "
                 f"{st['bp_iters']} iterations / {launches} launches")
    elif dominant == "k_frame":
        words = math.ceil(shots / 64)
        ops = FRAME_OPS_PER_CX_WORD * info["gates_2q"] * words * args.steps / launches
        model = f"{FRAME_OPS_PER_CX_WORD} lane-ops per CX per 64-shot word"
    else:
        ops = float("nan")
        model = "no model"
    achieved = ops / avg_s / 1e12
    roofline = dict(bound="alu", achieved=achieved, peak=VALU_PEAK_TOPS, unit="TOP/s",
                    frac=achieved / VALU_PEAK_TOPS, traffic=traffic_bytes(w.name, dominant), kernel=dominant,
                    avg_launch_ms=avg_s * 1e3, model=model)
    # the sampler's frame kernel against the same VALU peak (frame bit-operations only)
    sample_roofline = None
    if "k_frame" in kern:
        fl, fms = kern["k_frame"]
        words = math.ceil(shots / 64)
        f_ops = FRAME_OPS_PER_CX_WORD * info["gates_2q"] * words * args.steps / fl
        f_ach = f_ops / (fms / fl / 1e3) / 1e12
        sample_roofline = dict(bound="alu", kernel="k_frame", achieved=f_ach, peak=VALU_PEAK_TOPS, unit="TOP/s",
                               frac=f_ach / VALU_PEAK_TOPS, traffic=traffic_bytes(w.name, "k_frame"),
                               avg_launch_ms=fms / fl,
                               model=f"{FRAME_OPS_PER_CX_WORD} lane-ops per CX per 64-shot word x "
                                     f"{info['gates_2q']} CX x {words} words")
    # the whole sampler (event generation and frames) against the frame + RNG model
    sample_roofline_rng = None
    if sample_ms:
        ev = info["events_per_mshot"] / 1e6
        w_shot = (FRAME_OPS_PER_CX_WORD * info["gates_2q"] / 64.0 + info["noise_sites"] / 4096.0 * PHILOX_OPS_PER_DRAW
                  + ev * (2 * PHILOX_OPS_PER_DRAW + GAP_SEARCH_OPS + EVENT_APPLY_OPS))
        s_ach = w_shot * total / (sample_ms / 1e3) / 1e12
        sample_roofline_rng = dict(bound="alu", kernels="k_event_count + k_scan_* + k_event_write + k_frame",
                                   achieved=s_ach, peak=VALU_PEAK_TOPS, unit="TOP/s", frac=s_ach / VALU_PEAK_TOPS,
                                   model=(f"{w_shot:.1f} lane-ops per shot: {FRAME_OPS_PER_CX_WORD} per CX per 64 "
                                          f"shots, {PHILOX_OPS_PER_DRAW} per Philox draw (one per site and "
                                          f"4096-shot block, two per event), {GAP_SEARCH_OPS} per gap search, "
                                          f"{EVENT_APPLY_OPS} per event applied; {ev:.2f} events per shot"))
    ler = errors / total
    out = {
        "metric": "shots/sec (sample+BP-OSD decode) on 1 MI355X at matched logical error rate",
        "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64+f32", "data": "synthetic (seeded Philox circuit noise)",
        "config": {"workload": w.name, "description": w.description, "shots_per_step": shots,
                   "bp_iters": w.bp_iters, "osd": "OSD-0", "detectors": dem.rows, "dem_columns": dem.cols,
                   "dem_edges": dem.edges},
        "sample_shots_per_s": total / (sample_ms / 1e3) if sample_ms else None,
        "decode_shots_per_s": total / (decode_ms / 1e3) if decode_ms else None,
        "logical_error_rate": ler, "ler_sigma": math.sqrt(max(ler * (1 - ler), 0) / total),
        "osd_rate": st["osd"] / max(st["shots"], 1), "bp_iters_mean": st["bp_iters"] / max(st["shots"], 1),
        "kernels_ms": {n: round(v[1] / v[0], 4) for n, v in sorted(kern.items())},
        "roofline": roofline,
        "sample_roofline": sample_roofline,
        "sample_roofline_rng": sample_roofline_rng,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
