"""Train and evaluate the convolutional surrogate of 16 RK4 steps.

    python -m paper_1203_1263_amd.surrogate_train [--trajectories 200] [--iters 32000]

Workload: 2D defocusing NLSE on 256^2 (h = 0.25, a = 1, s = -1, V = 0, MSD
boundaries, 2SHOC, FP32 with compensation, dt = 0.8 of the linear bound).
Initial conditions: 2-8 seeded singly charged vortices on a unit background.

1. Data: the batched integrator advances all trajectories together; after a
   burn-in of 160 steps, 101 snapshots are taken 16 steps apart, giving
   100 (psi(t), psi(t + 16 dt)) pairs per trajectory.  Trajectories are split
   90/5/5 into train / validation / test.
2. Training: Adam on the mean squared error of the 16-step increment, with
   the library's forward / backward / optimiser kernels.  With pushforward
   p > 0, after the first 30% of the iterations a fraction p of the
   iterations trains on the network's own prediction of psi(t + 16 dt)
   (forward pass plus MSD projection, no gradient through it) as input and
   psi(t + 32 dt) as target, so the network also sees inputs carrying its
   own one-block error (the pushforward trick of learned simulators).
3. Evaluation on test trajectories: relative L2 distance to RK4 after each
   of 1 .. 10 surrogate blocks (and the largest block count within 1e-2), relative mass and energy drift per block, fallback
   count of the guarded advance (mass drift tolerance 1e-3), and the time of
   one block (surrogate + mass check) against 16 RK4 steps at batch 1 and
   batch 64.

Every numerical step runs in libnlse; PyTorch holds device memory.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as wl
from .nlse import Batch, Grid, Surrogate, nlse_dt_max

N, H_STEP, A, S_NL = 256, 0.25, 1.0, -1.0
BLOCK = 16
# algorithmic flops of one forward pass per pixel: 2 per multiply-add over
# the six 3x3 layers with their real channel counts (2-48-48-48-48-48-2)
FLOP_PER_PIXEL = 2 * 9 * (2 * 48 + 4 * 48 * 48 + 48 * 2)
# HBM bytes of one forward pass per pixel, each activation read and written
# once in the kernels' layout: packing (8 B complex64 in, 16 B = 8 BF16
# channels out), layer 1 (16 in, 96 out), layers 2-5 (96 in, 96 out), layer 6
# (96 in, plus the 8 B input field read and the 8 B prediction written).
# At 169 344 flop per 1016 B (167 flop/B) the pass sits below the BF16 ridge
# (2.5 PFLOP/s / 8 TB/s = 312 flop/B): it is HBM-bound.
BYTES_PER_PIXEL = (8 + 16) + (16 + 96) + 4 * (96 + 96) + (96 + 8 + 8)


class _P:
    def __init__(self, psi0):
        self.psi0, self.h, self.a, self.s, self.V, self.order, self.bc = psi0, H_STEP, A, S_NL, None, 4, "msd"


def dt_default():
    return 0.8 * nlse_dt_max(2, 4, H_STEP, A)


def generate(ntraj: int, npairs: int = 100, burn: int = 160, seed_index: int = 4):
    """Snapshots [ntraj, npairs + 1, N, N] complex64 on the device."""
    import torch
    g = wl.rng(seed_index)
    probs = [_P(wl.surrogate_ic(g, N, H_STEP)) for _ in range(ntraj)]
    dt = dt_default()
    b = Batch(probs, [dt] * ntraj, compensated=True)
    b.autotune()  # any configuration gives the same bits; this one is fastest
    snaps = torch.empty((ntraj, npairs + 1, N, N), dtype=torch.complex64, device="cuda")
    pool = b.pool.view(ntraj, N, N)
    b.step(burn)
    for k in range(npairs + 1):
        snaps[:, k].copy_(pool)
        if k < npairs:
            b.step(BLOCK)
    b.status()
    torch.cuda.synchronize()
    b.close()
    return snaps


def init_params(seed: int = 0, last_scale: float = 0.1):
    """He-normal weights (last layer scaled down), zero biases, as float32."""
    g = np.random.Generator(np.random.PCG64(seed))
    chans = (2, 48, 48, 48, 48, 48, 2)
    out = []
    for l in range(6):
        cout, cin = chans[l + 1], chans[l]
        W = g.standard_normal((cout, cin, 3, 3)) * math.sqrt(2.0 / (cin * 9))
        if l == 5:
            W *= last_scale
        out += [W.ravel(), np.zeros(cout)]
    return np.concatenate(out).astype(np.float32)


def train(snaps, train_idx, iters: int, batch: int = 32, lr: float = 1e-3, seed: int = 0, log_every: int = 100,
          pushforward: float = 0.0):
    import torch
    params = torch.from_numpy(init_params(seed)).cuda()
    m = Surrogate(N, N, max(batch, 64), H_STEP, params=params)
    g = np.random.Generator(np.random.PCG64(seed + 1))
    npairs = snaps.shape[1] - 1
    x = torch.empty((batch, N, N), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    x0 = torch.empty_like(x)
    hist = []
    t0 = time.perf_counter()
    for it in range(iters):
        tr = g.choice(train_idx, size=batch)
        push = pushforward > 0 and it >= 0.3 * iters and g.random() < pushforward
        k = g.integers(0, npairs - (1 if push else 0), size=batch)
        ti = torch.from_numpy(tr).cuda()
        ki = torch.from_numpy(k).cuda()
        if push:
            x0.copy_(snaps[ti, ki])
            m.forward(x0, x)
            m.project_msd(x0, x)
            y.copy_(snaps[ti, ki + 2])
        else:
            x.copy_(snaps[ti, ki])
            y.copy_(snaps[ti, ki + 1])
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / iters)) + 1e-5
        want = (it % log_every == 0) or it == iters - 1
        loss = m.train_step(x, y, lr_t, want_loss=want)
        if want:
            hist.append((it, loss))
            print(f"train it {it} loss {loss:.4e} lr {lr_t:.2e} {time.perf_counter() - t0:.1f}s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return m, params, hist, time.perf_counter() - t0


def _rel(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def evaluate(m, snaps, test_idx):
    """Relative L2 to RK4 after 1 .. 10 blocks (from each test trajectory's
    first snapshot), the largest block count within 1e-2, and the one-block
    error and mass drift over the trajectories."""
    import torch
    out = {}
    x0 = snaps[test_idx, 0].contiguous()
    y = x0
    curve = []
    for k in range(1, 11):
        pred = m.forward(y)
        m.project_msd(y, pred)
        y = pred
        curve.append(_rel(y, snaps[test_idx, k]))
    out["rel_l2_after_1_blocks"] = curve[0]
    out["rel_l2_after_10_blocks"] = curve[-1]
    out["rel_l2_after_k_blocks"] = curve
    n_ok = 0  # leading blocks whose error stays within 1e-2
    for e in curve:
        if e > 1e-2:
            break
        n_ok += 1
    out["blocks_within_1e-2"] = n_ok
    # one-block errors from every snapshot of the test trajectories
    errs, drifts = [], []
    for k in range(0, snaps.shape[1] - 1, 10):
        xk = snaps[test_idx, k].contiguous()
        pk = m.forward(xk)
        m.project_msd(xk, pk)
        errs.append(_rel(pk, snaps[test_idx, k + 1]))
        mi = np.array(m.field_mass(xk))
        mo = np.array(m.field_mass(pk))
        drifts.append(float(np.max(np.abs(mo - mi) / mi)))
    out["rel_l2_one_block_mean"] = float(np.mean(errs))
    out["mass_drift_per_block_max"] = float(np.max(drifts))
    return out


def guarded_advance(m, snaps, test_idx, nblocks: int = 10, tol: float = 1e-3):
    """Guarded advance of each test trajectory: fallback count and error."""
    import torch
    dt = dt_default()
    fb, errs = 0, []
    for t in test_idx:
        psi = snaps[t, 0].clone()
        g = Grid(psi, H_STEP, A, S_NL)
        fb += m.advance(g, 4, "msd", dt, nblocks, tol)
        torch.cuda.synchronize()
        errs.append(_rel(psi, snaps[t, nblocks]))
        g.close()
    return {"fallbacks": fb, "blocks": nblocks * len(test_idx), "rel_l2_guarded": float(np.mean(errs))}


def _time(fn, reps: int):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def speedup(m, snaps, batch: int):
    """Time of one block (surrogate forward, MSD projection and mass check,
    one library call) vs 16 RK4 steps of the fastest integrator
    configuration: at batch 1 the faster of an autotuned four-pass grid and
    an autotuned stage-pair grid, at larger batches the autotuned batched
    integrator (tile, grid size, four passes or stage pairs)."""
    import torch
    dt = dt_default()
    fields = snaps[:batch, 0].contiguous()
    out = torch.empty_like(fields)

    def surrogate_block():
        m.block(fields, out)  # forward, MSD projection and masses in one pass (synchronises)

    if batch == 1:
        t_rk, rk_config = None, None
        for pairs in (False, True):
            psi = fields[0].clone()
            g = Grid(psi, H_STEP, A, S_NL, compensated=True, fused_pairs=pairs)
            g.autotune(4, "msd", dt)

            def rk4_block():
                g.step(dt, BLOCK, order=4, bc="msd")
            t = _time(rk4_block, 10)
            if t_rk is None or t < t_rk:
                t_rk, rk_config = t, {"stage_pairs": pairs, "tile": list(g.tile(4))}
            g.close()
    else:
        probs = [_P(fields[i].cpu().numpy()) for i in range(batch)]
        b = Batch(probs, [dt] * batch, compensated=True)
        b.autotune()

        def rk4_block():
            b.step(BLOCK)
        t_rk = _time(rk4_block, 10)
        tx, ty, wg, pairs = b.config()
        rk_config = {"stage_pairs": bool(pairs), "tile": [tx, ty], "wg_per_cu": wg}
        b.close()
    # inference kernels the block takes: the whole-network kernel for small
    # batches, one kernel per layer otherwise (the same bits either way)
    path = "fused" if batch <= m.fused_max_batch() else "layers"
    t_sg = _time(surrogate_block, 10)
    t_fwd = _time(lambda: m.forward(fields, out), 10)
    extra = {}
    if path == "fused":
        m.set_path("layers")
        extra = {"ms_surrogate_block_layers": _time(surrogate_block, 10),
                 "ms_forward_layers": _time(lambda: m.forward(fields, out), 10)}
        m.set_path("auto")
    fwd_flop = FLOP_PER_PIXEL * batch * N * N
    fwd_bytes = BYTES_PER_PIXEL * batch * N * N
    return {"batch": batch, "ms_rk4_16_steps": t_rk, "rk4_config": rk_config, "ms_surrogate_block": t_sg,
            "speedup": t_rk / t_sg, "path": path, **extra,
            "ms_forward": t_fwd, "forward_tflops": fwd_flop / (t_fwd * 1e-3) / 1e12,
            "forward_gbs": fwd_bytes / (t_fwd * 1e-3) / 1e9}


def run(ntraj: int = 200, iters: int = 32000, batch: int = 32, lr: float = 1e-3, seed: int = 0,
        pushforward: float = 0.0):
    import torch
    t0 = time.perf_counter()
    snaps = generate(ntraj)
    t_gen = time.perf_counter() - t0
    print(f"generated {ntraj} trajectories in {t_gen:.1f}s", file=sys.stderr, flush=True)
    perm = np.random.Generator(np.random.PCG64(77)).permutation(ntraj)
    ntr, nva = int(round(0.9 * ntraj)), max(1, int(round(0.05 * ntraj)))
    train_idx, val_idx, test_idx = perm[:ntr], perm[ntr:ntr + nva], perm[ntr + nva:]
    if len(test_idx) == 0:
        test_idx = val_idx
    m, params, hist, t_train = train(snaps, train_idx, iters, batch=batch, lr=lr, seed=seed,
                                     pushforward=pushforward)
    res = {"trajectories": ntraj, "pairs": ntraj * (snaps.shape[1] - 1), "iters": iters, "batch": batch,
           "pushforward": pushforward,
           "seconds_generate": t_gen, "seconds_train": t_train, "loss_first": hist[0][1], "loss_last": hist[-1][1]}
    ti = torch.from_numpy(np.asarray(test_idx)).cuda()
    res.update(evaluate(m, snaps, ti))
    res.update(guarded_advance(m, snaps, test_idx[:4]))
    res["speedup_b1"] = speedup(m, snaps, 1)
    res["speedup_b64"] = speedup(m, snaps, min(64, ntraj, m.max_batch))
    res["loss_history"] = hist
    return res, m, params


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trajectories", type=int, default=200)
    ap.add_argument("--iters", type=int, default=32000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--pushforward", type=float, default=0.0)
    a = ap.parse_args()
    res, _, _ = run(a.trajectories, a.iters, a.batch, a.lr, pushforward=a.pushforward)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
