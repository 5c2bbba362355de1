"""Chunk-size study (Sec. "Chunk-size Limitations").

The paper integrates 1000 RK4 steps and hands the field back to the host
every `chunk` steps; the slowdown of a chunk size is the run time with a
single chunk of 1000 steps divided by the run time with that chunk size
(1 = no cost, 0.5 = twice as slow).  It measures grids of about 10^3, 10^4,
10^5 and 10^6 points in 1D, 2D (floor(sqrt N)^2) and 3D (floor(cbrt N)^3),
CD2 and 2SHOC, single and double precision.

Here two ways of handing frames back are timed on the same grids:

* ``overlap``: :meth:`Grid.run_frames` (``nlse_run_frames``): after each
  chunk the field is copied device to device into a staging half, and a
  second stream copies it to pinned host memory while the next chunk runs;
* ``sync``: the pattern of a host loop that waits for each chunk and copies
  the field into pageable host memory before launching the next one.

Run time is host wall time around the whole 1000-step run (after a warm-up
run of the same shape, which also captures the step graphs).  Fields are
smooth synthetic data with MSD boundaries; their values do not affect the
timing.  Frames that would need more than ``max_frame_bytes`` of host memory
are skipped and reported as such.

    python -m paper_1203_1263_amd.chunk_study [--out results.json] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

STEPS = 1000
CHUNKS = (1, 2, 5, 10, 20, 50, 100, 200, 500, 1000)
SIZES = (1_000, 10_000, 100_000, 1_000_000)


def grid_shape(ndim: int, n: int):
    if ndim == 1:
        return (n,)
    side = int(math.floor(n ** (1.0 / ndim) + 1e-9))
    return (side,) * ndim


def _field(shape, dtype):
    import torch
    from . import workloads as wl
    u = 1.0 + 0.2 * wl.random_field(shape, 17, smooth=2.0)
    return torch.from_numpy(np.ascontiguousarray(u, dtype=np.complex64 if dtype == "f32" else np.complex128)).cuda()


def measure(ndim: int, n: int, order: int, dtype: str, chunks=CHUNKS, max_frame_bytes: float = 2 * 2 ** 30):
    """Wall time (s) of STEPS steps for each chunk size, both modes."""
    import torch
    from .nlse import Grid, nlse_dt_max
    shape = grid_shape(ndim, n)
    npts = int(np.prod(shape))
    h, a, s = 0.25, 1.0, -1.0
    dt = 0.5 * nlse_dt_max(ndim, order, h, a)
    psi = _field(shape, dtype)
    g = Grid(psi, h, a, s)
    fb = psi.numel() * psi.element_size()
    ok = [c for c in chunks if (STEPS // c) * fb <= max_frame_bytes]
    nmax = max(STEPS // c for c in ok)
    pinned = torch.empty((nmax,) + shape, dtype=psi.dtype, pin_memory=True)
    pageable = torch.empty((nmax,) + shape, dtype=psi.dtype)
    out = {"ndim": ndim, "shape": list(shape), "npts": npts, "order": order, "dtype": dtype,
           "frame_bytes": fb, "overlap": {}, "sync": {}, "skipped": [c for c in chunks if c not in ok]}
    for c in ok:
        nf = STEPS // c
        for mode in ("overlap", "sync"):
            best = float("inf")
            for rep in range(3):  # rep 0 warms up (graph capture, page faults)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "overlap":
                    g.run_frames(dt, c, nf, order=order, bc="msd", out=pinned)
                else:
                    for j in range(nf):
                        g.step(dt, c, order=order, bc="msd")
                        pageable[j].copy_(psi)  # waits for the chunk, then a blocking copy
                torch.cuda.synchronize()
                if rep:
                    best = min(best, time.perf_counter() - t0)
            out[mode][c] = best
    g.close()
    return out


def d2h_rate(nbytes: int = 256 * 2 ** 20, reps: int = 5):
    """Device-to-host copy rate (GB/s) into pinned and pageable memory."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    out = {}
    for name, dst in (("pinned", torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)),
                      ("pageable", torch.empty(nbytes, dtype=torch.uint8))):
        dst.copy_(src)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            dst.copy_(src)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        out[name] = nbytes / best / 1e9
    return out


def slowdowns(r):
    """Slowdown factors, each relative to the mode's own single-chunk run."""
    res = {}
    for mode in ("overlap", "sync"):
        t = r[mode]
        ref = t.get(STEPS)
        res[mode] = {c: (ref / v if ref else None) for c, v in t.items()}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=None, help="write all timings as JSON here")
    ap.add_argument("--quick", action="store_true", help="2D FP32 2SHOC only")
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("chunk_study needs a GPU")
    combos = [(d, o, p) for d in (1, 2, 3) for o in (2, 4) for p in ("f32", "f64")]
    if args.quick:
        combos = [(2, 4, "f32")]
    rate = d2h_rate()
    print(f"device-to-host copy of 256 MiB: pinned {rate['pinned']:.1f} GB/s, "
          f"pageable {rate['pageable']:.1f} GB/s", flush=True)
    results = [{"d2h_GBps": rate}]
    for d, o, p in combos:
        for n in SIZES:
            r = measure(d, n, o, p)
            sd = slowdowns(r)
            results.append(r)
            line = " ".join(f"{c}:{sd['overlap'][c]:.2f}/{sd['sync'][c]:.2f}" for c in sorted(sd["overlap"]))
            print(f"{d}D {'CD2' if o == 2 else '2SHOC'} {p} N={r['npts']:>8} "
                  f"t1000={r['overlap'][STEPS] * 1e3:7.2f} ms  slowdown overlap/sync {line}"
                  + (f"  (skipped chunks {r['skipped']})" if r["skipped"] else ""), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(results, f, indent=1)


if __name__ == "__main__":
    main()
