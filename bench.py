"""Benchmark: grid-point RK4 updates per second of the fused HIP integrator.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 3D Gross-Pitaevskii problem on a 256^3 grid (harmonic trap,
Thomas-Fermi background with a vortex ring), FP32 storage with the
compensated FP64 final RK4 combination, 2SHOC Laplacian, MSD boundaries.  A
"step" is one full RK4 step (four fused stage kernels) over the whole grid;
inputs are resident in HBM before the timed region starts.

Prints one JSON line with the throughput, the roofline position of the stage
kernel (algorithmic bytes / measured time against 8 TB/s HBM), a CPU
baseline (the FP64 oracle timed on a bounded sample on the host cores) and a
summary of the learned surrogate (trained here on trajectories of the
integrator: error against RK4 after 1..10 blocks of 16 steps and speedup over
16 RK4 steps at batch 1 and 64).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per grid point per RK4 step (each array touched once
# per stage; halos and the 2SHOC temporary stay on chip):
#   S1: r Psi 8, r V 4, w acc 8, w U1 8                      = 28
#   S2: r U1 8, r V 4, r Psi 8, r/w acc 16, w U2 8           = 44
#   S3: same as S2                                           = 44
#   S4 (compensated): r U3 8, V 4, acc 8, Psi_hi 8, Psi_lo 8,
#       w Psi_hi 8, w Psi_lo 8                               = 52
BYTES_PER_PT_STEP = {"compensated": 168, "plain": 144}
# HBM bytes per stage launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
# (FETCH_SIZE scaled by 2.0, WRITE_SIZE by 1.0 against a plain 1 GiB copy) for
# the compensated 256^3 run with tile (32, 8, 16); reported only for that
# configuration.
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA
MEASURED_TRAFFIC = {("compensated", 256, (32, 8, 16)): 756.3e6}
# HBM bytes per point-step of the batched workload's kernel, from FETCH_SIZE /
# WRITE_SIZE counters, keyed by (tile, stage pairs, mode)
BATCH_TRAFFIC = {((32, 32), True, "compensated"): 84.4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256, help="grid extent per axis (default 256)")
    ap.add_argument("--plain", action="store_true", help="plain FP32 (no compensation)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-problems summary")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate summary (trajectory generation, training and timing, ~15 s)")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of each CPU-baseline run (0: 40 on all cores, 6 on one)")
    ap.add_argument("--tile", type=int, nargs=3, default=None, metavar=("TX", "TY", "CZ"),
                    help="stage tile (default: the library's default tile)")
    ap.add_argument("--autotune", action="store_true", help="let the autotuner pick the tile")
    ap.add_argument("--workload", choices=["ring3d", "batch2d", "surrogate"], default="ring3d",
                    help="ring3d: 3D GPE at n^3 (default); batch2d: 512 uneven 2D problems in one launch; "
                         "surrogate: train the 16-step surrogate and time it against RK4")
    ap.add_argument("--trajectories", type=int, default=200, help="surrogate: trajectories of 100 pairs")
    ap.add_argument("--iters", type=int, default=32000, help="surrogate: Adam iterations")
    ap.add_argument("--cpu-child", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def copy_probe():
    """A plain device-to-device copy of exactly 1 GiB, 10 times: reference
    for the FETCH_SIZE / WRITE_SIZE counters and for achievable bandwidth."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * (1 << 30) * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    print(json.dumps({"copy_probe_bytes_each_way": 1 << 30, "copies": 10, "GB/s": gbs}), flush=True)


def bench_batch(args):
    print(json.dumps(run_batch(args, args.steps)), flush=True)


def run_batch(args, steps):
    """512 independent 2D problems (sizes 64..512 per axis, CD2 or 2SHOC,
    per-problem a, s, V, dt), compensated FP32, advanced together by the
    persistent graph-captured kernel; `steps` steps in one launch."""
    import torch
    from paper_1203_1263_amd import workloads as wl
    from paper_1203_1263_amd.nlse import Batch, nlse_dt_max
    probs = wl.batch2d()
    dts = [0.8 * nlse_dt_max(2, p.order, p.h, p.a) for p in probs]
    b = Batch(probs, dts, compensated=not args.plain)
    t_tune = time.perf_counter()
    b.autotune()  # tile and workgroups per CU for this batch (fields untouched)
    t_tune = time.perf_counter() - t_tune
    b.step(steps)  # capture + warm-up with the timed step count
    b.status()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    b.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.status()
    gpu_s = ev0.elapsed_time(ev1) * 1e-3
    info = b.info()
    npts = info["points"]
    tx, ty, wg, pairs = b.config()
    bpp = BYTES_PER_PT_STEP["plain" if args.plain else "compensated"]
    # bytes the chosen pass structure moves per point-step: two stage-pair
    # passes keep the intermediate stages on chip (28 + 52 B compensated,
    # 28 + 36 B plain); the roofline stays against the four-pass figure
    kbpp = (80 if not args.plain else 64) if pairs else bpp
    achieved = npts * bpp * steps / gpu_s / 1e9
    tb = BATCH_TRAFFIC.get(((tx, ty), bool(pairs), "plain" if args.plain else "compensated"))
    traffic = tb * npts * steps if tb else None  # HBM bytes of the timed launch
    out = {"metric": "grid-point RK4 updates/s (512 batched 2D problems)", "value": npts * steps / wall,
           "unit": "grid-point RK4 updates/s", "n_gpus": 1, "steps": steps, "warmup": steps,
           "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" + ("" if args.plain else "+f64-compensated"),
           "data": "synthetic",
           "config": {"workload": "batch2d_512_problems_persistent_graph", "points": npts,
                      "workgroups": info["workgroups"], "items": info["items"],
                      "tile": [tx, ty], "wg_per_cu": wg, "stage_pairs": bool(pairs), "autotuned": True,
                      "autotune_s": t_tune},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                        "kernel": "batch2d_pair_kernel (persistent, stage pairs)" if pairs
                        else "batch2d_kernel (persistent, all stages)",
                        "bytes_per_point_step": bpp, "kernel_bytes_per_point_step": kbpp,
                        "kernel_GBps": npts * kbpp * steps / gpu_s / 1e9}}
    b.close()
    return out


def bench_surrogate(args):
    """Generate trajectories with the integrator, train the surrogate on them
    with the library's kernels, and report its accuracy and its speedup over
    16 RK4 steps at batch 1 and 64."""
    from paper_1203_1263_amd import surrogate_train as st
    res, _, _ = st.run(args.trajectories, args.iters)
    hist = res.pop("loss_history")
    out = {"metric": "surrogate speedup over 16 RK4 steps (2D 256^2 vortex fields)",
           "value": res["speedup_b64"]["speedup"], "unit": "x", "n_gpus": 1, "steps": args.iters,
           "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16 (fp32 accumulate)", "data": "synthetic (trajectories of the FP32 2SHOC integrator)",
           "config": {"workload": "surrogate_256^2_2shoc_msd", "trajectories": args.trajectories},
           # 167 flop/B is below the BF16 ridge (312 flop/B): the forward pass is
           # HBM-bound; the MFMA rate is reported beside it
           "roofline": {"bound": "hbm", "achieved": res["speedup_b64"]["forward_gbs"], "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": res["speedup_b64"]["forward_gbs"] / HBM_PEAK_GBS,
                        "traffic": None, "bytes_per_pixel": st.BYTES_PER_PIXEL,
                        "mfma_tflops": res["speedup_b64"]["forward_tflops"], "mfma_peak_tflops": BF16_PEAK_TFLOPS,
                        "kernel": f"surrogate forward (pack + 6 conv3x3 MFMA launches), batch {res['speedup_b64']['batch']}"},
           "surrogate": res, "loss_history_every_100": hist}
    print(json.dumps(out), flush=True)


def _cpu_info():
    """Host CPU description: model name, logical CPUs this process may use,
    physical cores (distinct core ids per socket)."""
    model, phys = None, set()
    cur = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if cur:
                        phys.add((cur.get("physical id"), cur.get("core id")))
                    cur = {}
                    continue
                k, v = (t.strip() for t in line.split(":", 1))
                cur[k] = v
                if k == "model name" and model is None:
                    model = v
        if cur:
            phys.add((cur.get("physical id"), cur.get("core id")))
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": nproc, "physical_cores": len(phys) or None}


def _oracle_child(threads, steps, n):
    """Run the oracle in a child process with its own OpenMP settings (the
    thread count is fixed when the OpenMP runtime starts); returns
    (point-updates/s, seconds, steps)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), OMP_PROC_BIND="close", OMP_PLACES="cores")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", str(steps), "--n", str(n)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_child(steps, n):
    """Child of cpu_baseline: time the FP64 oracle on the bench workload."""
    import oracle
    from paper_1203_1263_amd import workloads as wl
    prob = wl.ring3d(shape=(n, n, n), h=0.1 * 256 / n)
    dt = 0.8 * oracle.dt_max(3, 4, prob.h, prob.a)
    t0 = time.perf_counter()
    oracle.rk4(prob.psi0, prob.h, prob.a, prob.s, dt, steps, V=prob.V, order=prob.order, bc=prob.bc)
    el = time.perf_counter() - t0
    print(json.dumps({"rate": prob.npts * steps / el, "seconds": el, "steps": steps}), flush=True)


def cpu_baseline(steps_hint, n):
    """Time the FP64 oracle as it stands on a bounded sample of the bench
    workload (256^3, 2SHOC + MSD), once on one thread and once on all the
    cores this host gives the job (OMP_NUM_THREADS if set, else its physical
    cores), each in a child process with OMP_PROC_BIND=close."""
    info = _cpu_info()
    share = int(os.environ.get("OMP_NUM_THREADS", 0) or 0)
    threads = share if share > 0 else (info["physical_cores"] or info["nproc"])
    many = _oracle_child(threads, steps_hint if steps_hint > 0 else 40, n)
    one = _oracle_child(1, steps_hint if steps_hint > 0 else 6, n)
    shape = f"{n}x{n}x{n} grid, 2SHOC+MSD, FP64"
    return {"value": many["rate"], "unit": "grid-point RK4 updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{shape}, {many['steps']} RK4 steps on {threads} OpenMP threads "
                      f"(OMP_PROC_BIND=close), {many['seconds']:.1f} s",
            "single_core": {"value": one["rate"], "cores": 1,
                            "sample": f"{shape}, {one['steps']} RK4 steps on 1 thread, {one['seconds']:.1f} s"},
            **info}


def main():
    args = parse()
    if args.cpu_child:
        cpu_child(args.cpu_child, args.n)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "batch2d":
        bench_batch(args)
        return
    if args.workload == "surrogate":
        bench_surrogate(args)
        return
    import torch
    from paper_1203_1263_amd import workloads as wl
    from paper_1203_1263_amd.nlse import Grid, nlse_dt_max, NLSE_2SHOC

    comp = not args.plain
    n = args.n
    h = 0.1 * 256 / n
    prob = wl.ring3d(shape=(n, n, n), h=h)
    dt = 0.8 * nlse_dt_max(3, 4, h, prob.a)
    psi = torch.from_numpy(prob.psi0.astype(np.complex64)).cuda()
    V = torch.from_numpy(prob.V.astype(np.float32)).cuda()
    stream = torch.cuda.current_stream()
    g = Grid(psi, h, prob.a, prob.s, V=V, compensated=comp, stream=stream)
    if args.tile:
        g.set_tile(NLSE_2SHOC, args.tile)
    elif args.autotune:
        g.autotune(NLSE_2SHOC, "msd", dt)
    tile = g.tile(NLSE_2SHOC)
    # warm-up: the timed call's own step count first, so every graph it
    # replays is captured and instantiated before the timed region
    g.step(dt, args.steps, order=NLSE_2SHOC, bc="msd")
    g.step(dt, args.warmup, order=NLSE_2SHOC, bc="msd")
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    g.step(dt, args.steps, order=NLSE_2SHOC, bc="msd")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)

    M, E = g.mass_energy(NLSE_2SHOC, "msd")
    npts = prob.npts
    value = npts * args.steps / wall
    bpp = BYTES_PER_PT_STEP["compensated" if comp else "plain"]
    launches = 4 * args.steps
    avg_launch_s = gpu_ms * 1e-3 / launches
    bytes_per_launch = npts * bpp / 4.0
    achieved = bytes_per_launch / avg_launch_s / 1e9
    out = {
        "metric": "grid-point RK4 updates/s (3D 2SHOC FP32, 256^3)",
        "value": value,
        "unit": "grid-point RK4 updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" + ("+f64-compensated" if comp else ""),
        "data": "synthetic",
        "config": {"workload": f"ring3d_{n}^3_2shoc_msd_{'compensated' if comp else 'plain'}_fp32",
                   "grid": [n, n, n], "h": h, "a": prob.a, "s": prob.s, "dt": dt,
                   "tile": list(tile), "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": MEASURED_TRAFFIC.get(("compensated" if comp else "plain", n, tuple(tile))),
                     "kernel": "stage3d_kernel<float,2SHOC,MSD>",
                     "bytes_per_point_step": bpp,
                     "avg_launch_us": avg_launch_s * 1e6},
        "mass": M, "energy": E,
    }
    g.close()
    del psi, V
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, n)
    if not args.no_batch:
        out["batch2d"] = batch_summary(args)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_summary(args)
    print(json.dumps(out), flush=True)


def batch_summary(args):
    """The batched workload in short (512 uneven 2D problems, autotuned,
    50 steps in one launch)."""
    r = run_batch(args, 50)
    keep = ("value", "unit", "ms_per_step", "steps")
    out = {k: r[k] for k in keep}
    out["config"] = {k: r["config"][k] for k in ("points", "tile", "wg_per_cu", "stage_pairs", "autotune_s")}
    out["roofline"] = {k: r["roofline"][k] for k in ("achieved", "frac", "traffic", "bytes_per_point_step",
                                                     "kernel_bytes_per_point_step", "kernel_GBps", "kernel")}
    return out


def surrogate_summary(args):
    """The learned-surrogate workload in short: generate its trajectories
    with the batched integrator, train it with the library's kernels, and
    report its error against RK4 and its speedup over 16 RK4 steps."""
    from paper_1203_1263_amd import surrogate_train as st
    res, m, _ = st.run(args.trajectories, args.iters)
    m.close()
    keep = ("trajectories", "pairs", "iters", "seconds_generate", "seconds_train", "rel_l2_after_1_blocks",
            "rel_l2_after_10_blocks", "rel_l2_after_k_blocks", "blocks_within_1e-2", "rel_l2_one_block_mean",
            "mass_drift_per_block_max", "fallbacks", "blocks", "rel_l2_guarded")
    out = {k: res[k] for k in keep}
    for b in ("speedup_b1", "speedup_b64"):
        out[b] = {k: res[b][k] for k in ("batch", "ms_rk4_16_steps", "rk4_config", "ms_surrogate_block", "speedup",
                                         "path", "ms_surrogate_block_layers") if k in res[b]}
    # the speedup holds for as many blocks as stay within the 1e-2 error bar
    out["speedup_within_1e-2"] = {"blocks": res["blocks_within_1e-2"],
                                  "batch_1": res["speedup_b1"]["speedup"], "batch_64": res["speedup_b64"]["speedup"]}
    out["forward_b64"] = {"TFLOP/s": res["speedup_b64"]["forward_tflops"], "GB/s": res["speedup_b64"]["forward_gbs"]}
    return out


if __name__ == "__main__":
    main()
