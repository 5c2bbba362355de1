"""Thin Python binding of libnlse (the C ABI declared in include/nlse.h).

Argument marshalling only: every step of the integrator runs in the HIP
kernels of ``libnlse.so``.  PyTorch provides device memory and streams.  If
the library is missing the import fails loudly -- there is no CPU fallback.

Raw entry points keep the C names (``nlse_create_grid``, ``nlse_step_rk4``,
...).  :class:`Grid` bundles a field, its workspace and potential tensors.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlse.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nlse.h")

NLSE_OK = 0
NLSE_EINVAL = -1
NLSE_ENOMEM = -2
NLSE_EDEVICE = -3
NLSE_EUNSTABLE = -4
NLSE_EUNSUPPORTED = -5
NLSE_F32, NLSE_F64 = 0, 1
NLSE_CD2, NLSE_2SHOC = 2, 4
NLSE_BC_DIRICHLET, NLSE_BC_MSD, NLSE_BC_L0 = 0, 1, 2
NLSE_COMPENSATED = 0x1
NLSE_SG_PATH_AUTO, NLSE_SG_PATH_LAYERS, NLSE_SG_PATH_FUSED = 0, 1, 2
NLSE_NO_GRAPH = 0x2
NLSE_FUSED_PAIRS = 0x4

BC = {"dirichlet": NLSE_BC_DIRICHLET, "msd": NLSE_BC_MSD, "l0": NLSE_BC_L0}


class SimDesc(ctypes.Structure):
    """nlse_sim_desc of include/nlse.h."""
    _fields_ = [("ndim", ctypes.c_int), ("dims", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("a", ctypes.c_double), ("s", ctypes.c_double), ("dt", ctypes.c_double),
                ("order", ctypes.c_int), ("bc", ctypes.c_int), ("psi_offset", ctypes.c_int64),
                ("v_offset", ctypes.c_int64)]


class NLSEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libnlse.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with "
                          "`python -m paper_1203_1263_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    sig = {
        "nlse_dt_max": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
        "nlse_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "nlse_last_error": (ctypes.c_char_p, []),
        "nlse_workspace_bytes": (ctypes.c_int, [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_uint,
                                                ctypes.POINTER(ctypes.c_size_t)]),
        "nlse_create_grid": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, i64p, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_uint,
                                            vp, vp, ctypes.c_size_t, vp]),
        "nlse_set_potential": (ctypes.c_int, [vp, vp]),
        "nlse_step_rk4": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int64]),
        "nlse_mass_energy": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, dp, dp]),
        "nlse_mass_energy_noalloc": (ctypes.c_int, [ctypes.c_int, i64p, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                    vp, vp, vp, dp, dp]),
        "nlse_run_frames": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                           ctypes.c_int64, vp, vp, ctypes.c_size_t]),
        "nlse_get_state": (ctypes.c_int, [vp, vp]),
        "nlse_set_state": (ctypes.c_int, [vp, vp]),
        "nlse_autotune": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double]),
        "nlse_get_tile": (ctypes.c_int, [vp, ctypes.c_int, ip]),
        "nlse_get_stage_pairs": (ctypes.c_int, [vp, ctypes.c_int, ip]),
        "nlse_set_tile": (ctypes.c_int, [vp, ctypes.c_int, ip]),
        "nlse_destroy_grid": (ctypes.c_int, [vp]),
        "nlse_batch_workspace_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(SimDesc), ctypes.c_int,
                                                      ctypes.c_uint, ctypes.POINTER(ctypes.c_size_t)]),
        "nlse_batch_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(SimDesc),
                                             ctypes.c_int, ctypes.c_uint, vp, ctypes.c_size_t, vp,
                                             ctypes.c_size_t, vp, ctypes.c_size_t, vp]),
        "nlse_batch_step_rk4": (ctypes.c_int, [vp, ctypes.c_int64]),
        "nlse_batch_mass_energy": (ctypes.c_int, [vp, dp, dp]),
        "nlse_batch_status": (ctypes.c_int, [vp]),
        "nlse_batch_info": (ctypes.c_int, [vp, i64p]),
        "nlse_batch_set_config": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "nlse_batch_get_config": (ctypes.c_int, [vp, ip]),
        "nlse_batch_autotune": (ctypes.c_int, [vp]),
        "nlse_batch_destroy": (ctypes.c_int, [vp]),
        "nlse_surrogate_param_count": (ctypes.c_int, []),
        "nlse_surrogate_workspace_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                          ctypes.POINTER(ctypes.c_size_t)]),
        "nlse_surrogate_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_double, vp, vp, ctypes.c_size_t, vp]),
        "nlse_surrogate_refresh": (ctypes.c_int, [vp]),
        "nlse_surrogate_forward": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "nlse_surrogate_loss_grad": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp, dp]),
        "nlse_surrogate_train_step": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, ctypes.c_float, dp]),
        "nlse_surrogate_field_mass": (ctypes.c_int, [vp, vp, ctypes.c_int, dp]),
        "nlse_surrogate_project_msd": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "nlse_surrogate_block": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, ctypes.c_int, dp]),
        "nlse_surrogate_advance": (ctypes.c_int, [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                  ctypes.c_int64, ctypes.c_double, i64p]),
        "nlse_surrogate_set_path": (ctypes.c_int, [vp, ctypes.c_int]),
        "nlse_surrogate_fused_max_batch": (ctypes.c_int, [vp]),
        "nlse_surrogate_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def header_symbols(path: str = HEADER):
    """Names of the functions declared in a public header (for export checks)."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nlse_[a-z0-9_]+)\s*\(", txt)))


def _check(rc: int, what: str):
    if rc != NLSE_OK:
        lib = load_library()
        raise NLSEError(rc, f"{what}: {lib.nlse_last_error().decode()}")


# ---------------------------------------------------------------- raw entry points

def nlse_dt_max(ndim: int, order: int, h: float, a: float) -> float:
    return load_library().nlse_dt_max(ndim, order, h, a)


def nlse_workspace_bytes(ndim: int, dims, dtype: int, flags: int = 0) -> int:
    lib = load_library()
    d = (ctypes.c_int64 * 3)(*dims)
    out = ctypes.c_size_t(0)
    _check(lib.nlse_workspace_bytes(ndim, d, dtype, flags, ctypes.byref(out)), "nlse_workspace_bytes")
    return out.value


def nlse_create_grid(ndim, dims, h, a, s, dtype, flags, psi_ptr, work_ptr, work_bytes, stream_ptr):
    lib = load_library()
    g = ctypes.c_void_p()
    d = (ctypes.c_int64 * 3)(*dims)
    _check(lib.nlse_create_grid(ctypes.byref(g), ndim, d, h, a, s, dtype, flags, psi_ptr, work_ptr,
                                work_bytes, stream_ptr), "nlse_create_grid")
    return g


def nlse_set_potential(g, V_ptr):
    _check(load_library().nlse_set_potential(g, V_ptr), "nlse_set_potential")


def nlse_step_rk4(g, order: int, bc: int, dt: float, nsteps: int):
    _check(load_library().nlse_step_rk4(g, order, bc, dt, nsteps), "nlse_step_rk4")


def nlse_run_frames(g, order: int, bc: int, dt: float, chunk: int, nframes: int, frames_host_ptr,
                    stage_ptr, stage_bytes: int):
    _check(load_library().nlse_run_frames(g, order, bc, dt, chunk, nframes, frames_host_ptr, stage_ptr,
                                          stage_bytes), "nlse_run_frames")


def nlse_mass_energy(g, order: int, bc: int) -> Tuple[float, float]:
    m, e = ctypes.c_double(), ctypes.c_double()
    _check(load_library().nlse_mass_energy(g, order, bc, ctypes.byref(m), ctypes.byref(e)),
           "nlse_mass_energy")
    return m.value, e.value


def nlse_mass_energy_noalloc(ndim: int, dims, h: float, a: float, s: float, dtype: int, order: int, bc: int,
                             psi_ptr: int, v_ptr: Optional[int], stream_ptr: Optional[int]) -> Tuple[float, float]:
    d = (ctypes.c_int64 * 3)(*dims)
    m, e = ctypes.c_double(), ctypes.c_double()
    _check(load_library().nlse_mass_energy_noalloc(ndim, d, h, a, s, dtype, order, bc, psi_ptr, v_ptr, stream_ptr,
                                                   ctypes.byref(m), ctypes.byref(e)),
           "nlse_mass_energy_noalloc")
    return m.value, e.value


def nlse_get_state(g, lo_ptr):
    _check(load_library().nlse_get_state(g, lo_ptr), "nlse_get_state")


def nlse_set_state(g, lo_ptr):
    _check(load_library().nlse_set_state(g, lo_ptr), "nlse_set_state")


def nlse_autotune(g, order: int, bc: int, dt: float):
    _check(load_library().nlse_autotune(g, order, bc, dt), "nlse_autotune")


def nlse_get_tile(g, order: int):
    t = (ctypes.c_int * 3)()
    _check(load_library().nlse_get_tile(g, order, t), "nlse_get_tile")
    return tuple(t)


def nlse_set_tile(g, order: int, tile):
    t = (ctypes.c_int * 3)(*tile)
    _check(load_library().nlse_set_tile(g, order, t), "nlse_set_tile")


def nlse_get_stage_pairs(g, order: int) -> bool:
    on = ctypes.c_int(0)
    _check(load_library().nlse_get_stage_pairs(g, order, ctypes.byref(on)), "nlse_get_stage_pairs")
    return bool(on.value)


def nlse_destroy_grid(g):
    _check(load_library().nlse_destroy_grid(g), "nlse_destroy_grid")


def nlse_batch_workspace_bytes(descs, dtype: int, flags: int = 0) -> int:
    arr = (SimDesc * len(descs))(*descs)
    out = ctypes.c_size_t(0)
    _check(load_library().nlse_batch_workspace_bytes(len(descs), arr, dtype, flags, ctypes.byref(out)),
           "nlse_batch_workspace_bytes")
    return out.value


def nlse_batch_create(descs, dtype, flags, psi_ptr, psi_elems, v_ptr, v_elems, work_ptr, work_bytes,
                      stream_ptr):
    arr = (SimDesc * len(descs))(*descs)
    b = ctypes.c_void_p()
    _check(load_library().nlse_batch_create(ctypes.byref(b), len(descs), arr, dtype, flags, psi_ptr,
                                            psi_elems, v_ptr, v_elems, work_ptr, work_bytes, stream_ptr),
           "nlse_batch_create")
    return b


def nlse_batch_step_rk4(b, nsteps: int):
    _check(load_library().nlse_batch_step_rk4(b, nsteps), "nlse_batch_step_rk4")


def nlse_batch_mass_energy(b, nsims: int):
    m = (ctypes.c_double * nsims)()
    e = (ctypes.c_double * nsims)()
    _check(load_library().nlse_batch_mass_energy(b, m, e), "nlse_batch_mass_energy")
    return list(m), list(e)


def nlse_batch_status(b):
    _check(load_library().nlse_batch_status(b), "nlse_batch_status")


def nlse_batch_info(b):
    info = (ctypes.c_int64 * 4)()
    _check(load_library().nlse_batch_info(b, info), "nlse_batch_info")
    return {"workgroups": info[0], "items": info[1], "points": info[2], "graphs": info[3]}


def nlse_batch_set_config(b, tx: int, ty: int, wg_per_cu: int, pairs: int = 0):
    _check(load_library().nlse_batch_set_config(b, tx, ty, wg_per_cu, int(pairs)), "nlse_batch_set_config")


def nlse_batch_get_config(b) -> Tuple[int, int, int, int]:
    c = (ctypes.c_int * 4)()
    _check(load_library().nlse_batch_get_config(b, c), "nlse_batch_get_config")
    return c[0], c[1], c[2], c[3]


def nlse_batch_autotune(b):
    _check(load_library().nlse_batch_autotune(b), "nlse_batch_autotune")


def nlse_batch_destroy(b):
    _check(load_library().nlse_batch_destroy(b), "nlse_batch_destroy")


def nlse_surrogate_param_count() -> int:
    return load_library().nlse_surrogate_param_count()


def nlse_surrogate_workspace_bytes(H: int, W: int, max_batch: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().nlse_surrogate_workspace_bytes(H, W, max_batch, ctypes.byref(out)),
           "nlse_surrogate_workspace_bytes")
    return out.value


def nlse_surrogate_create(H, W, max_batch, h, params_ptr, work_ptr, work_bytes, stream_ptr):
    m = ctypes.c_void_p()
    _check(load_library().nlse_surrogate_create(ctypes.byref(m), H, W, max_batch, h, params_ptr, work_ptr,
                                                work_bytes, stream_ptr), "nlse_surrogate_create")
    return m


def nlse_surrogate_refresh(m):
    _check(load_library().nlse_surrogate_refresh(m), "nlse_surrogate_refresh")


def nlse_surrogate_forward(m, psi_in_ptr, psi_out_ptr, batch):
    _check(load_library().nlse_surrogate_forward(m, psi_in_ptr, psi_out_ptr, batch), "nlse_surrogate_forward")


def nlse_surrogate_loss_grad(m, psi_in_ptr, tgt_ptr, batch, grad_ptr=None, want_loss=True):
    loss = ctypes.c_double(0.0)
    _check(load_library().nlse_surrogate_loss_grad(m, psi_in_ptr, tgt_ptr, batch, grad_ptr,
                                                   ctypes.byref(loss) if want_loss else None),
           "nlse_surrogate_loss_grad")
    return loss.value


def nlse_surrogate_train_step(m, psi_in_ptr, tgt_ptr, batch, lr, want_loss=True):
    loss = ctypes.c_double(0.0)
    _check(load_library().nlse_surrogate_train_step(m, psi_in_ptr, tgt_ptr, batch, lr,
                                                    ctypes.byref(loss) if want_loss else None),
           "nlse_surrogate_train_step")
    return loss.value


def nlse_surrogate_field_mass(m, psi_ptr, batch):
    out = (ctypes.c_double * batch)()
    _check(load_library().nlse_surrogate_field_mass(m, psi_ptr, batch, out), "nlse_surrogate_field_mass")
    return list(out)


def nlse_surrogate_block(m, psi_in, psi_out, batch: int, project_msd: bool = True):
    """Forward, MSD projection and masses of one surrogate block in one pass."""
    out = (ctypes.c_double * batch)()
    _check(load_library().nlse_surrogate_block(m, psi_in, psi_out, batch, 1 if project_msd else 0, out),
           "nlse_surrogate_block")
    return list(out)


def nlse_surrogate_project_msd(m, psi_in_ptr, psi_out_ptr, batch):
    _check(load_library().nlse_surrogate_project_msd(m, psi_in_ptr, psi_out_ptr, batch),
           "nlse_surrogate_project_msd")


def nlse_surrogate_advance(m, g, order, bc, dt, nblocks, drift_tol):
    nf = ctypes.c_int64(0)
    _check(load_library().nlse_surrogate_advance(m, g, order, bc, dt, nblocks, drift_tol, ctypes.byref(nf)),
           "nlse_surrogate_advance")
    return nf.value


def nlse_surrogate_set_path(m, path: int):
    _check(load_library().nlse_surrogate_set_path(m, path), "nlse_surrogate_set_path")


def nlse_surrogate_fused_max_batch(m) -> int:
    r = load_library().nlse_surrogate_fused_max_batch(m)
    _check(min(r, 0), "nlse_surrogate_fused_max_batch")
    return r


def nlse_surrogate_destroy(m):
    _check(load_library().nlse_surrogate_destroy(m), "nlse_surrogate_destroy")


# ---------------------------------------------------------------- convenience objects

class Grid:
    """A field on the GPU plus the library grid that integrates it.

    ``psi`` is a complex64 (FP32) or complex128 (FP64) CUDA tensor of shape
    (Nz, Ny, Nx) / (Ny, Nx) / (Nx,), updated in place.
    """

    def __init__(self, psi, h: float, a: float, s: float, V=None, compensated: bool = False,
                 stream=None, fused_pairs: bool = False, graph: bool = True):
        import torch
        load_library()
        if not psi.is_cuda:
            raise ValueError("psi must be a device tensor")
        if psi.dtype == torch.complex64:
            self.dtype = NLSE_F32
            self.rdtype = torch.float32
        elif psi.dtype == torch.complex128:
            self.dtype = NLSE_F64
            self.rdtype = torch.float64
        else:
            raise ValueError("psi must be complex64 or complex128")
        if not psi.is_contiguous():
            raise ValueError("psi must be contiguous")
        self.psi = psi
        self.ndim = psi.dim()
        self.dims = list(reversed(psi.shape)) + [1] * (3 - self.ndim)
        self.h, self.a, self.s = float(h), float(a), float(s)
        self.flags = ((NLSE_COMPENSATED if compensated else 0) | (NLSE_FUSED_PAIRS if fused_pairs else 0)
                      | (0 if graph else NLSE_NO_GRAPH))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nbytes = nlse_workspace_bytes(self.ndim, self.dims, self.dtype, self.flags)
        self.work = torch.empty(nbytes + 256, dtype=torch.uint8, device=psi.device)
        off = (-self.work.data_ptr()) % 256
        self.work_ptr = self.work.data_ptr() + off
        self.work_bytes = nbytes
        self._g = nlse_create_grid(self.ndim, self.dims, self.h, self.a, self.s, self.dtype, self.flags,
                                   psi.data_ptr(), self.work_ptr, nbytes, self.stream.cuda_stream)
        self.V = None
        if V is not None:
            self.set_potential(V)

    def set_potential(self, V):
        if V is None:
            self.V = None
            nlse_set_potential(self._g, None)
            return
        if V.dtype != self.rdtype or tuple(V.shape) != tuple(self.psi.shape) or not V.is_contiguous():
            raise ValueError("V must be a contiguous real tensor of psi's shape and precision")
        self.V = V
        nlse_set_potential(self._g, V.data_ptr())

    def step(self, dt: float, nsteps: int, order: int = NLSE_2SHOC, bc="msd"):
        nlse_step_rk4(self._g, order, BC[bc] if isinstance(bc, str) else bc, dt, nsteps)

    def run_frames(self, dt: float, chunk: int, nframes: int, order: int = NLSE_2SHOC, bc="msd",
                   out=None, pinned: bool = True):
        """Advance nframes * chunk steps; returns the field after every chunk
        as a host tensor of shape (nframes, *psi.shape) (pinned unless
        ``pinned=False`` or ``out`` is given)."""
        import torch
        if out is None:
            out = torch.empty((nframes,) + tuple(self.psi.shape), dtype=self.psi.dtype, pin_memory=pinned)
        if out.is_cuda or not out.is_contiguous() or out.dtype != self.psi.dtype or \
                out.numel() < nframes * self.psi.numel():
            raise ValueError("out must be a contiguous host tensor of nframes fields")
        if getattr(self, "_stage", None) is None:
            self._stage = torch.empty(2 * self.psi.numel(), dtype=self.psi.dtype, device=self.psi.device)
        nlse_run_frames(self._g, order, BC[bc] if isinstance(bc, str) else bc, dt, chunk, nframes,
                        out.data_ptr() if nframes else None, self._stage.data_ptr(),
                        self._stage.numel() * self._stage.element_size())
        return out

    def mass_energy(self, order: int = NLSE_CD2, bc="dirichlet"):
        return nlse_mass_energy(self._g, order, BC[bc] if isinstance(bc, str) else bc)

    def get_state(self):
        import torch
        lo = torch.empty_like(self.psi)
        nlse_get_state(self._g, lo.data_ptr())
        return lo

    def set_state(self, lo=None):
        nlse_set_state(self._g, None if lo is None else lo.data_ptr())
        self._lo_keep = lo

    def autotune(self, order: int, bc, dt: float):
        nlse_autotune(self._g, order, BC[bc] if isinstance(bc, str) else bc, dt)

    def tile(self, order: int):
        return nlse_get_tile(self._g, order)

    def set_tile(self, order: int, tile):
        nlse_set_tile(self._g, order, tile)

    def stage_pairs(self, order: int) -> bool:
        """Whether steps of this order run as stage pairs now."""
        return nlse_get_stage_pairs(self._g, order)

    def close(self):
        if self._g:
            nlse_destroy_grid(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent 2D problems advanced by one persistent launch.

    ``problems``: sequence of objects with ``psi0`` (2D complex array),
    ``h``, ``a``, ``s``, ``V`` (array or None), ``order``, ``bc`` and a time
    step given by ``dts[j]``.  Fields live in one device pool (``self.pool``);
    ``field(j)`` returns a view of problem j.
    """

    def __init__(self, problems, dts, dtype: str = "f32", compensated: bool = False,
                 graph: bool = True, stream=None):
        import numpy as np
        import torch
        load_library()
        self.np_c = np.complex64 if dtype == "f32" else np.complex128
        self.np_r = np.float32 if dtype == "f32" else np.float64
        self.tc = torch.complex64 if dtype == "f32" else torch.complex128
        self.tr = torch.float32 if dtype == "f32" else torch.float64
        self.dtype = NLSE_F32 if dtype == "f32" else NLSE_F64
        self.flags = (NLSE_COMPENSATED if compensated else 0) | (0 if graph else NLSE_NO_GRAPH)
        self.shapes = []
        descs = []
        poff = voff = 0
        vparts, pparts = [], []
        for p, dt in zip(problems, dts):
            psi0 = np.asarray(p.psi0)
            if psi0.ndim != 2:
                raise ValueError("batches hold 2D problems")
            ny, nx = psi0.shape
            d = SimDesc()
            d.ndim = 2
            d.dims[0], d.dims[1], d.dims[2] = nx, ny, 1
            d.h, d.a, d.s, d.dt = float(p.h), float(p.a), float(p.s), float(dt)
            d.order = int(p.order)
            d.bc = BC[p.bc] if isinstance(p.bc, str) else int(p.bc)
            d.psi_offset = poff
            if p.V is not None:
                d.v_offset = voff
                vparts.append(np.asarray(p.V, dtype=self.np_r).ravel())
                voff += nx * ny
            else:
                d.v_offset = -1
            pparts.append(psi0.astype(self.np_c).ravel())
            self.shapes.append((ny, nx, poff))
            poff += nx * ny
            descs.append(d)
        self.descs = descs
        self.pool = torch.from_numpy(np.concatenate(pparts)).cuda()
        self.vpool = torch.from_numpy(np.concatenate(vparts)).cuda() if vparts else None
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nbytes = nlse_batch_workspace_bytes(descs, self.dtype, self.flags)
        self.work = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.pool.device)
        wptr = self.work.data_ptr() + ((-self.work.data_ptr()) % 256)
        self._b = nlse_batch_create(descs, self.dtype, self.flags, self.pool.data_ptr(), poff,
                                    self.vpool.data_ptr() if self.vpool is not None else None,
                                    voff, wptr, nbytes, self.stream.cuda_stream)

    def field(self, j):
        ny, nx, off = self.shapes[j]
        return self.pool[off:off + nx * ny].view(ny, nx)

    def step(self, nsteps: int):
        nlse_batch_step_rk4(self._b, nsteps)

    def mass_energy(self):
        return nlse_batch_mass_energy(self._b, len(self.descs))

    def status(self):
        nlse_batch_status(self._b)

    def info(self):
        return nlse_batch_info(self._b)

    def set_config(self, tx: int, ty: int, wg_per_cu: int, pairs: bool = False):
        nlse_batch_set_config(self._b, tx, ty, wg_per_cu, 1 if pairs else 0)

    def config(self):
        """(tile x-width, tile y-height, persistent workgroups per CU,
        1 if a step runs as two stage-pair passes else 0)."""
        return nlse_batch_get_config(self._b)

    def autotune(self):
        nlse_batch_autotune(self._b)

    def close(self):
        if self._b:
            nlse_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """The convolutional surrogate of 16 RK4 steps on H x W complex64 fields.

    ``params`` is a float32 device tensor of ``nlse_surrogate_param_count()``
    values (per layer W (Cout, Cin, 3, 3) then b); it is updated in place by
    :meth:`train_step`.
    """

    def __init__(self, H: int, W: int, max_batch: int, h: float, params=None, stream=None):
        import torch
        load_library()
        n = nlse_surrogate_param_count()
        if params is None:
            params = torch.zeros(n, dtype=torch.float32, device="cuda")
        if params.dtype != torch.float32 or params.numel() != n or not params.is_cuda:
            raise ValueError(f"params must be a float32 device tensor of {n} values")
        self.params = params
        self.H, self.W, self.max_batch = H, W, max_batch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nbytes = nlse_surrogate_workspace_bytes(H, W, max_batch)
        self.work = torch.empty(nbytes + 256, dtype=torch.uint8, device=params.device)
        wptr = self.work.data_ptr() + ((-self.work.data_ptr()) % 256)
        self._m = nlse_surrogate_create(H, W, max_batch, h, params.data_ptr(), wptr, nbytes,
                                        self.stream.cuda_stream)

    def _check_fields(self, psi):
        import torch
        if psi.dtype != torch.complex64 or not psi.is_contiguous() or tuple(psi.shape[-2:]) != (self.H, self.W):
            raise ValueError("fields must be contiguous complex64 [batch, H, W]")
        return psi.shape[0] if psi.dim() == 3 else 1

    def refresh(self):
        nlse_surrogate_refresh(self._m)

    def forward(self, psi, out=None):
        import torch
        b = self._check_fields(psi)
        out = torch.empty_like(psi) if out is None else out
        nlse_surrogate_forward(self._m, psi.data_ptr(), out.data_ptr(), b)
        return out

    def loss_grad(self, psi, target):
        import torch
        b = self._check_fields(psi)
        grad = torch.empty_like(self.params)
        loss = nlse_surrogate_loss_grad(self._m, psi.data_ptr(), target.data_ptr(), b, grad.data_ptr())
        return loss, grad

    def train_step(self, psi, target, lr: float, want_loss: bool = True):
        b = self._check_fields(psi)
        return nlse_surrogate_train_step(self._m, psi.data_ptr(), target.data_ptr(), b, lr, want_loss)

    def field_mass(self, psi):
        b = self._check_fields(psi)
        return nlse_surrogate_field_mass(self._m, psi.data_ptr(), b)

    def block(self, psi_in, psi_out, project_msd: bool = True):
        """One surrogate block (forward, MSD projection, masses) in one pass;
        returns the masses of psi_out."""
        b = self._check_fields(psi_in)
        return nlse_surrogate_block(self._m, psi_in.data_ptr(), psi_out.data_ptr(), b, project_msd)

    def project_msd(self, psi_in, psi_out):
        b = self._check_fields(psi_in)
        nlse_surrogate_project_msd(self._m, psi_in.data_ptr(), psi_out.data_ptr(), b)

    def set_path(self, path):
        """Inference kernels: "auto", "layers" (one kernel per layer) or
        "fused" (all six layers in one kernel); the same bits either way."""
        nlse_surrogate_set_path(self._m, {"auto": NLSE_SG_PATH_AUTO, "layers": NLSE_SG_PATH_LAYERS,
                                          "fused": NLSE_SG_PATH_FUSED}[path] if isinstance(path, str) else path)

    def fused_max_batch(self) -> int:
        return nlse_surrogate_fused_max_batch(self._m)

    def advance(self, grid, order, bc, dt, nblocks, drift_tol):
        return nlse_surrogate_advance(self._m, grid._g, order, BC[bc] if isinstance(bc, str) else bc, dt,
                                      nblocks, drift_tol)

    def close(self):
        if self._m:
            nlse_surrogate_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
