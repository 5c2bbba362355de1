"""FP64 CPU oracle for the NLSEmagic RK4 integrator (arXiv:1203.1263).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, independent
reference the GPU library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product package never does.  It shares no code with the GPU
path: the C source ``nlse_oracle.c`` is compiled here with ``gcc -O2
-ffp-contract=off -fopenmp`` and called through ctypes.

Functions (each cites the passage of the paper it follows, in the C source):

* :func:`dt_max` -- Eqs. stblincd / stblin2shoc.
* :func:`rhs` -- F(Psi) of Eq. RK4 with the CD2 / 2SHOC Laplacian and the
  Dirichlet / MSD / Laplacian-zero boundary forms (Sec. "Boundary
  conditions").
* :func:`laplacian` -- the scheme Laplacian alone at interior points.
* :func:`rk4` -- classic RK4 (Eq. RK4) with its four slopes k_1..k_4.
* :func:`mass_energy` -- standard NLSE invariants (not defined by the paper).

Arrays are complex128 numpy arrays of shape ``(Nz, Ny, Nx)``, ``(Ny, Nx)`` or
``(Nx,)`` (x fastest), i.e. interleaved complex with linear index
``x + Nx*(y + Ny*z)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nlse_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC = {"dirichlet": 0, "msd": 1, "l0": 2}
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_long)
    lib.orc_dt_max.restype = ctypes.c_double
    lib.orc_dt_max.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    common = [ctypes.c_int, lp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp,
              ctypes.c_int, ctypes.c_int]
    lib.orc_rhs.argtypes = common + [dp, dp]
    lib.orc_laplacian.argtypes = common + [dp, dp]
    lib.orc_rk4.argtypes = common + [ctypes.c_double, ctypes.c_long, dp]
    lib.orc_mass_energy.argtypes = common + [dp, dp]
    for f in (lib.orc_rhs, lib.orc_laplacian, lib.orc_rk4, lib.orc_mass_energy):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _dims(psi: np.ndarray):
    ndim = psi.ndim
    if ndim < 1 or ndim > 3:
        raise ValueError("psi must be 1-, 2- or 3-dimensional")
    n = list(reversed(psi.shape)) + [1] * (3 - ndim)  # (Nx, Ny, Nz)
    return ndim, (ctypes.c_long * 3)(*n)


def _cplx(psi) -> np.ndarray:
    return np.ascontiguousarray(psi, dtype=np.complex128)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vptr(V, shape):
    if V is None:
        return None, ctypes.POINTER(ctypes.c_double)()
    V = np.ascontiguousarray(V, dtype=np.float64)
    if V.shape != shape:
        raise ValueError("V must have the shape of psi")
    return V, _ptr(V)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def dt_max(ndim: int, order: int, h: float, a: float) -> float:
    """Linear RK4 stability bound (Eq. stblincd; 3/4 of it for 2SHOC, Eq. stblin2shoc)."""
    return _load().orc_dt_max(int(ndim), int(order), float(h), float(a))


def rhs(psi, h, a, s, V=None, order=2, bc="dirichlet") -> np.ndarray:
    """F(psi) = i[a L psi + (s|psi|^2 - V) psi] with boundary forms."""
    lib = _load()
    u = _cplx(psi)
    ndim, n = _dims(u)
    Vk, vp = _vptr(V, u.shape)
    F = np.zeros_like(u)
    _check(lib.orc_rhs(ndim, n, h, a, s, vp, order, BC[bc], _ptr(u), _ptr(F)), "rhs")
    return F


def laplacian(psi, h, a=1.0, s=0.0, V=None, order=2, bc="dirichlet") -> np.ndarray:
    """Scheme Laplacian at interior points (boundary entries are zero)."""
    lib = _load()
    u = _cplx(psi)
    ndim, n = _dims(u)
    Vk, vp = _vptr(V, u.shape)
    L = np.zeros_like(u)
    _check(lib.orc_laplacian(ndim, n, h, a, s, vp, order, BC[bc], _ptr(u), _ptr(L)),
           "laplacian")
    return L


def rk4(psi, h, a, s, dt, nsteps, V=None, order=2, bc="dirichlet") -> np.ndarray:
    """Advance ``nsteps`` classic RK4 steps (Eq. RK4); returns a new array."""
    lib = _load()
    u = _cplx(psi).copy()
    ndim, n = _dims(u)
    Vk, vp = _vptr(V, u.shape)
    _check(lib.orc_rk4(ndim, n, h, a, s, vp, order, BC[bc], float(dt), int(nsteps), _ptr(u)),
           "rk4")
    return u


def mass_energy(psi, h, a, s, V=None, order=2, bc="dirichlet"):
    """(M, E): M = h^d sum|psi|^2, E = h^d[sum_int -a Re(conj psi L psi) + sum V|psi|^2 - s/2 |psi|^4]."""
    lib = _load()
    u = _cplx(psi)
    ndim, n = _dims(u)
    Vk, vp = _vptr(V, u.shape)
    out = np.zeros(2)
    _check(lib.orc_mass_energy(ndim, n, h, a, s, vp, order, BC[bc], _ptr(u), _ptr(out)),
           "mass_energy")
    return float(out[0]), float(out[1])
