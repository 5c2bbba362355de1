"""Seeded synthetic inputs for the NLSE workloads.

This module only *generates inputs* (grids, initial conditions, potentials,
parameter draws).  It holds none of the integrator's arithmetic, so both the
GPU path and the CPU oracle can be fed from it.  Every generator is seeded
(NumPy PCG64) and deterministic.

Workloads (the paper uses analytic initial conditions only, Sec. "Example test
problems"; the shapes below follow those examples and the benchmark configs):

* ``soliton1d``  -- 1D bright soliton sqrt(2c/s) sech(sqrt(c/a) x) e^{ict},
  N=1024 on x in [-50, 50] (end points included), a=1, s=1, c=1.
* ``dark_soliton1d`` -- the paper's co-moving dark soliton (Eq. soliton).
* ``vortex2d``   -- product of singly charged dark vortices tanh(r_j) e^{i m_j theta_j}
  on a unit background (after Eq. exmp2Dvort, with the tanh core the paper
  uses as its approximate profile), 1024^2, h=0.25, s=-1.
* ``ring3d``     -- Thomas-Fermi background in a harmonic trap
  V = 0.5 sum w_d x_d^2 with an embedded vortex ring (after Eq. 3dvr1, with a
  tanh core, or with ``core="exact"`` the numerically exact vortex profile),
  256^3 and 87x87x203.
* ``ring3d_paper`` -- the paper's own 3D example (Eq. 3dvr1): the exact
  charge-1 vortex profile in the ring's cross-section on a unit background,
  V = 0, with the co-moving back-flow phase e^{i c z / (2a)}.
* ``vortex_profile`` -- the numerically exact radial profile of a dark
  vortex (Eq. exmp2Dvort), found by Newton's method.
* ``batch2d``    -- 512 independent 2D problems of uneven size with Gaussian
  random-field initial conditions and smooth random potentials.
* ``surrogate2d`` -- 256^2 fields with 2-8 random vortices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 1000


def rng(index: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator for workload ``index`` (seed 1000 + index)."""
    return np.random.Generator(np.random.PCG64([SEED_BASE + index, stream]))


@dataclass
class Problem:
    """One grid problem: field, potential and physical parameters."""
    name: str
    psi0: np.ndarray           # complex128, shape (Nz, Ny, Nx) / (Ny, Nx) / (Nx,)
    h: float
    a: float
    s: float
    V: Optional[np.ndarray]    # float64 of psi0.shape, or None (V = 0)
    order: int                 # 2 = CD2, 4 = 2SHOC
    bc: str                    # "dirichlet" | "msd"
    nsteps: int
    dt_fraction: float = 0.8   # dt = dt_fraction * linear stability bound
    meta: dict = field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return self.psi0.ndim

    @property
    def npts(self) -> int:
        return int(self.psi0.size)


def axis(n: int, h: float) -> np.ndarray:
    """Grid coordinates centred on 0: (i - (n-1)/2) h, i = 0..n-1."""
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * h


# ------------------------------------------------------------------ 1D

def soliton1d(n: int = 1024, L: float = 100.0, c: float = 1.0, a: float = 1.0,
              s: float = 1.0, order: int = 2, nsteps: int = 1000) -> Problem:
    """Bright soliton on [-L/2, L/2] with both end points on the grid."""
    h = L / (n - 1)
    x = -L / 2 + np.arange(n) * h
    psi = np.sqrt(2 * c / s) / np.cosh(np.sqrt(c / a) * x) + 0j
    return Problem("soliton1d", psi, h, a, s, None, order, "dirichlet", nsteps,
                   meta={"c": c, "x": x})


def soliton1d_exact(x: np.ndarray, t: float, c: float = 1.0, a: float = 1.0,
                    s: float = 1.0) -> np.ndarray:
    return np.sqrt(2 * c / s) / np.cosh(np.sqrt(c / a) * x) * np.exp(1j * c * t)


def dark_soliton1d_exact(x, t, a=1.0, s=-1.0, c=0.5, om=-1.0):
    """Eq. soliton: co-moving dark soliton (s < 0)."""
    amp = np.sqrt(abs(om / s))
    k = np.sqrt(abs(om) / (2 * a))
    ph = (c / (2 * a)) * x + (om - c * c / (4 * a)) * t
    return amp * np.tanh(k * (x - c * t)) * np.exp(1j * ph)


# ------------------------------------------------------------------ 2D vortices

def _vortex_centres(g: np.random.Generator, nv: int, box: float, min_dist: float, max_draws: int = 100000):
    pts: List[np.ndarray] = []
    draws = 0
    while len(pts) < nv:
        draws += 1
        if draws > max_draws:
            raise ValueError(f"cannot place {nv} centres {min_dist} apart in a box of half-width {box}")
        p = g.uniform(-box, box, size=2)
        if all(np.hypot(*(p - q)) >= min_dist for q in pts):
            pts.append(p)
    return np.array(pts)


# ------------------------------------------------------------------ exact vortex profile

def vortex_profile(m: int = 1, a: float = 1.0, rmax: float = 40.0, dr: float = 0.01, tol: float = 1e-11,
                   max_iter: int = 30):
    """Radial profile g of the stationary charge-m dark vortex on a unit
    background (Eq. exmp2Dvort with s = -1, V = 0, so Omega = -1):

        a (g'' + g'/r - m^2 g / r^2) + (1 - g^2) g = 0,   g(0) = 0,

    with g(rmax) = 1 - a m^2 / (2 rmax^2) (the far-field expansion).  At
    background density rho the profile is sqrt(rho) g(r sqrt(rho)).  Solved
    by Newton's method on a second-order finite-difference grid with a
    banded Jacobian (the paper finds the numerically exact profile with a
    Newton-Krylov solver).  Returns (r, g) on r = 0, dr, ..., rmax."""
    from scipy.linalg import solve_banded
    M = int(round(rmax / dr))
    r = np.arange(M + 1) * dr
    rj = r[1:M]
    gM = 1.0 - a * m * m / (2.0 * rmax * rmax)
    g = np.tanh(r / math.sqrt(2.0 * a)) ** abs(m)
    g[0], g[M] = 0.0, gM
    lo_c = a * (1.0 / dr ** 2 - 1.0 / (2.0 * rj * dr))
    up_c = a * (1.0 / dr ** 2 + 1.0 / (2.0 * rj * dr))
    for _ in range(max_iter):
        gj, gm, gp = g[1:M], g[0:M - 1], g[2:M + 1]
        F = lo_c * gm + up_c * gp + a * (-2.0 / dr ** 2 - m * m / rj ** 2) * gj + (1.0 - gj * gj) * gj
        ab = np.zeros((3, M - 1))
        ab[0, 1:] = up_c[:-1]
        ab[1, :] = a * (-2.0 / dr ** 2 - m * m / rj ** 2) + 1.0 - 3.0 * gj * gj
        ab[2, :-1] = lo_c[1:]
        delta = solve_banded((1, 1), ab, -F)
        g[1:M] += delta
        step = np.max(np.abs(delta))
        if step < tol:
            break
    if step > 1e-8:  # rounding keeps fine grids from reaching tol; a real failure is far above this
        raise RuntimeError("vortex profile: Newton did not converge")
    return r, g


def _core(rr: np.ndarray, profile, a: float, m: int = 1) -> np.ndarray:
    """Profile value at radii rr: interpolated inside the table, far-field
    expansion 1 - a m^2/(2 r^2) beyond it."""
    r, g = profile
    out = np.interp(rr, r, g)
    far = rr > r[-1]
    if np.any(far):
        out[far] = 1.0 - a * m * m / (2.0 * rr[far] ** 2)
    return out


def vortex_field(x: np.ndarray, y: np.ndarray, centres, charges, profile=None, a: float = 1.0) -> np.ndarray:
    """Product of charge-m_j vortices: tanh(r_j) cores, or with ``profile``
    (from :func:`vortex_profile`, same a) the exact cores."""
    X, Y = np.meshgrid(x, y, indexing="xy")  # shape (Ny, Nx), x fastest
    psi = np.ones_like(X, dtype=np.complex128)
    for (cx, cy), m in zip(centres, charges):
        dx, dy = X - cx, Y - cy
        r = np.hypot(dx, dy)
        core = np.tanh(r) if profile is None else _core(r, profile, a, abs(int(m)))
        psi *= core * np.exp(1j * m * np.arctan2(dy, dx))
    return psi


def vortex2d(n: int = 1024, h: float = 0.25, nv: int = 4, nsteps: int = 2000,
             index: int = 1, box: float = 64.0, min_dist: float = 8.0, core: str = "tanh") -> Problem:
    g = rng(index)
    centres = _vortex_centres(g, nv, min(box, 0.4 * n * h), min_dist)
    charges = g.choice([-1, 1], size=nv)
    x = axis(n, h)
    profile = vortex_profile(1, 1.0) if core == "exact" else None
    psi = vortex_field(x, x, centres, charges, profile=profile, a=1.0)
    return Problem("vortex2d", psi, h, 1.0, -1.0, None, 4, "msd", nsteps,
                   meta={"centres": centres, "charges": charges, "core": core})


# ------------------------------------------------------------------ 3D ring

def ring3d(shape=(256, 256, 256), h: float = 0.1, nsteps: int = 1000, index: int = 2,
           a: float = 0.5, s: float = -1.0, core: str = "tanh") -> Problem:
    """shape = (Nz, Ny, Nx).  Thomas-Fermi density rho = mu - V (mu = max V + 1)
    with a vortex ring of radius R around the z axis: u = (r_perp - R) + i z,
    psi = sqrt(rho) tanh(|u|/xi) u/|u|, xi = sqrt(a/mu); with core="exact"
    the tanh is replaced by the exact profile at density mu,
    g(|u| sqrt(mu)) (see :func:`vortex_profile`)."""
    g = rng(index)
    nz, ny, nx = shape
    w = g.uniform(0.01, 0.1, size=3)
    x, y, z = axis(nx, h), axis(ny, h), axis(nz, h)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    V = 0.5 * (w[0] * X * X + w[1] * Y * Y + w[2] * Z * Z)
    mu = float(V.max()) + 1.0
    rho = mu - V
    half_x, half_y = x[-1], y[-1]
    rmax = min(8.0, 0.75 * min(half_x, half_y))
    R = g.uniform(3.0, rmax)
    xi = math.sqrt(a / mu)
    u = (np.hypot(X, Y) - R) + 1j * Z
    au = np.abs(u)
    with np.errstate(invalid="ignore", divide="ignore"):
        ph = np.where(au > 0, u / np.where(au > 0, au, 1.0), 0.0)
    if core == "exact":
        prof = vortex_profile(1, a)
        cz = _core((au * math.sqrt(mu)).ravel(), prof, a).reshape(au.shape)
    else:
        cz = np.tanh(au / xi)
    psi = np.sqrt(rho) * cz * ph
    return Problem("ring3d", psi.astype(np.complex128), h, a, s, V, 4, "msd", nsteps,
                   meta={"w": w, "R": R, "mu": mu, "core": core})


def ring_velocity(d: float, a: float) -> float:
    """Asymptotic speed of a large vortex ring of radius d on a unit
    background of iPsi_t = -a Lap Psi + |Psi|^2 Psi: the classical
    (ln(8R/xi) - 0.615)/(2R) law of the defocusing NLSE in units with
    a = 1/2, carried to general a by x -> x sqrt(2a)."""
    return (a / d) * (math.log(8.0 * d / math.sqrt(2.0 * a)) - 0.615)


def ring3d_paper(shape=(64, 64, 64), h: float = 0.5, d: float = 5.0, a: float = 1.0,
                 nsteps: int = 1000) -> Problem:
    """The paper's 3D example (Eq. 3dvr1): psi = g(r, z) e^{i c z / (2a)},
    g the exact charge-1 vortex at (r = d, z = 0) of the r-z half-plane on a
    unit background, V = 0, s = -1, c the ring's asymptotic speed
    (:func:`ring_velocity`), MSD boundaries, 2SHOC."""
    nz, ny, nx = shape
    x, y, z = axis(nx, h), axis(ny, h), axis(nz, h)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    u = (np.hypot(X, Y) - d) + 1j * Z
    au = np.abs(u)
    with np.errstate(invalid="ignore", divide="ignore"):
        ph = np.where(au > 0, u / np.where(au > 0, au, 1.0), 0.0)
    prof = vortex_profile(1, a)
    g = _core(au.ravel(), prof, a).reshape(au.shape) * ph
    c = ring_velocity(d, a)
    psi = g * np.exp(1j * (c / (2.0 * a)) * Z)
    return Problem("ring3d_paper", psi.astype(np.complex128), h, a, -1.0, None, 4, "msd", nsteps,
                   meta={"d": d, "c": c})


# ------------------------------------------------------------------ batch

BATCH_SIZES = (64, 128, 192, 256, 384, 512)


def _gaussian_blur_noise(g, ny, nx, sigma_cells):
    noise = g.standard_normal((ny, nx)) + 1j * g.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (math.pi ** 2) * (sigma_cells ** 2) * (kx * kx + ky * ky))
    f = np.fft.ifft2(np.fft.fft2(noise) * filt)
    return f / np.sqrt(np.mean(np.abs(f) ** 2))


# Mass of the 2D ground state R of Laplacian(R) - R + R^3 = 0 (the Townes
# profile), 2 pi int R^2 r dr: the critical mass of the focusing cubic NLSE in
# 2D.  For i psi_t + a Lap psi + s |psi|^2 psi = 0 (s > 0) it scales to
# TOWNES_MASS * a / s; below it solutions exist for all time, above it they
# can collapse in finite time.
TOWNES_MASS = 11.7008965


def batch2d(nsims: int = 512, h: float = 0.25, nsteps: int = 500, index: int = 3,
            sizes=BATCH_SIZES) -> List[Problem]:
    """Independent 2D problems: Nx, Ny drawn independently from ``sizes``;
    a ~ U[0.5, 1], s ~ {-1, +1}, scheme ~ {CD2, 2SHOC}; V = sum of four
    Gaussians with amplitudes U[-1, 1] and widths U[0.05, 0.2] L_min; IC =
    complex white noise blurred by a Gaussian of 4 cells (correlation length
    4h), unit RMS, times exp(-r^2 / 2 sigma_e^2), sigma_e = L_min/8, scaled to
    max |psi|^2 = 1, and for focusing problems (s = +1) further down to at
    most half the critical mass TOWNES_MASS * a / s, so no problem collapses
    (above it the continuous solution can blow up in finite time, which an
    explicit integrator cannot follow).  Zero-ish edges, so Dirichlet
    boundaries."""
    g = rng(index)
    out = []
    for j in range(nsims):
        nx, ny = int(g.choice(sizes)), int(g.choice(sizes))
        a = float(g.uniform(0.5, 1.0))
        s = float(g.choice([-1.0, 1.0]))
        order = int(g.choice([2, 4]))
        x, y = axis(nx, h), axis(ny, h)
        X, Y = np.meshgrid(x, y, indexing="xy")
        Lmin = min(nx, ny) * h
        V = np.zeros_like(X)
        for _ in range(4):
            A = g.uniform(-1, 1)
            sig = g.uniform(0.05, 0.2) * Lmin
            cx, cy = g.uniform(x[0], x[-1]), g.uniform(y[0], y[-1])
            V += A * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * sig * sig))
        psi = _gaussian_blur_noise(g, ny, nx, 4.0)
        se = Lmin / 8.0
        psi = psi * np.exp(-(X * X + Y * Y) / (2 * se * se))
        psi = psi / np.sqrt(np.max(np.abs(psi) ** 2))
        if s > 0:
            mass, cap = h * h * float(np.sum(np.abs(psi) ** 2)), 0.5 * TOWNES_MASS * a / s
            if mass > cap:
                psi = psi * np.sqrt(cap / mass)
        out.append(Problem(f"batch{j}", psi, h, a, s, V, order, "dirichlet", nsteps))
    return out


# ------------------------------------------------------------------ surrogate

def surrogate_ic(g: np.random.Generator, n: int = 256, h: float = 0.25) -> np.ndarray:
    """2..8 random singly charged vortices, centres in the central half."""
    nv = int(g.integers(2, 9))
    half = 0.25 * n * h
    centres = _vortex_centres(g, nv, half, 2.0)
    charges = g.choice([-1, 1], size=nv)
    x = axis(n, h)
    return vortex_field(x, x, centres, charges)


def surrogate2d(index: int = 4, n: int = 256, h: float = 0.25) -> Problem:
    g = rng(index)
    return Problem("surrogate2d", surrogate_ic(g, n, h), h, 1.0, -1.0, None, 4, "msd", 16)


# ------------------------------------------------------------------ spectra for tests

def random_field(shape, index: int, stream: int = 0, smooth: float = 0.0) -> np.ndarray:
    """Complex random field (optionally Gaussian-smoothed over ``smooth`` cells)."""
    g = rng(index, stream)
    f = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    if smooth > 0:
        F = np.fft.fftn(f)
        k2 = sum(np.meshgrid(*[np.fft.fftfreq(n) ** 2 for n in shape], indexing="ij"))
        f = np.fft.ifftn(F * np.exp(-2 * math.pi ** 2 * smooth ** 2 * k2))
        f /= np.sqrt(np.mean(np.abs(f) ** 2))
    return f
