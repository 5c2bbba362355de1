"""Helpers shared by the GPU tests: run the HIP path on a seeded problem and
compare with oracle results."""
from __future__ import annotations

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def to_dev(arr, dtype: str):
    import torch
    if dtype == "f32":
        return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.complex64)).cuda()
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.complex128)).cuda()


def pot_dev(V, dtype: str):
    import torch
    if V is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(V, dtype=np.float32 if dtype == "f32" else np.float64)).cuda()


def run_gpu(psi0, h, a, s, dt, nsteps, V=None, order=4, bc="msd", dtype="f32",
            compensated=False, tile=None, autotune=False, return_grid=False, fused_pairs=False, graph=True):
    """Integrate on the GPU through the C ABI; returns the final field (numpy)."""
    import torch
    from paper_1203_1263_amd.nlse import Grid
    psi = to_dev(psi0, dtype)
    Vd = pot_dev(V, dtype)
    g = Grid(psi, h, a, s, V=Vd, compensated=compensated, fused_pairs=fused_pairs, graph=graph)
    if tile is not None:
        g.set_tile(order, tile)
    if autotune:
        g.autotune(order, bc, dt)
    g.step(dt, nsteps, order=order, bc=bc)
    torch.cuda.synchronize()
    out = psi.cpu().numpy().astype(np.complex128)
    if return_grid:
        return out, g
    g.close()
    return out
