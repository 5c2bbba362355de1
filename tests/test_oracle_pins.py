"""Pins of the FP64 CPU oracle to facts fixed by the paper and by mathematics.

None of these tests compares the oracle with itself or retypes its formulas:
each checks it against a printed value, a closed form, an exact discrete
solution, an invariant, a convergence rate, or an independent formula.
"""
import ctypes
import math
import os

import numpy as np
import pytest

import oracle
from paper_1203_1263_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def R4(z):
    """Stability polynomial of classic RK4 (fourth-order Taylor polynomial)."""
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


# ---------------------------------------------------------------- stability bound

def _read_dt_golden():
    rows = []
    with open(os.path.join(GOLDEN, "dt_max_paper.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            p = line.split()
            rows.append((int(p[0]), int(p[1]), float(p[2]), float(p[3]), float(p[4]),
                         float(p[5]), p[6]))
    return rows


@pytest.mark.parametrize("row", _read_dt_golden(), ids=lambda r: r[6][:40])
def test_dt_max_printed_values(row):
    ndim, order, h, a, printed, rtol, _ = row
    assert oracle.dt_max(ndim, order, h, a) == pytest.approx(printed, rel=rtol)


def test_rk4_imaginary_axis_limit():
    """|R(i theta)| = 1 exactly at theta = 2 sqrt 2 and > 1 beyond: with the
    largest CD2 / 2SHOC eigenvalue magnitudes 4da/h^2 and (16/3)da/h^2 this is
    the bound of Eqs. stblincd / stblin2shoc."""
    th = 2 * math.sqrt(2)
    assert abs(R4(1j * th)) == pytest.approx(1.0, abs=1e-14)
    assert abs(R4(1j * th * 1.001)) > 1.0
    assert abs(R4(1j * th * 0.999)) < 1.0
    for ndim in (1, 2, 3):
        for order, lam in ((2, 4.0), (4, 16.0 / 3.0)):
            h, a = 0.3, 0.7
            kmax = oracle.dt_max(ndim, order, h, a)
            assert kmax * lam * ndim * a / h ** 2 == pytest.approx(th, rel=1e-14)


# ---------------------------------------------------------------- exact discrete dispersion

def _lam(kappa_h, order):
    """Eigenvalue of the 1D scheme Laplacian times h^2 for mode kappa."""
    s2 = math.sin(kappa_h / 2) ** 2
    lam = -4 * s2
    if order == 4:
        lam *= 1 + s2 / 3
    return lam


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("bc", ["dirichlet", "l0"])
def test_dispersion_sine_dirichlet(ndim, order, bc):
    """s = V = 0, zero boundary values: a product of sines is an exact
    eigenmode of the scheme, so RK4 gives psi^n = R(i a k lambda)^n psi^0.
    With s = V = 0 the Laplacian-zero condition (Eqs. BCL0dt, BCL0lap) gives
    F_b = 0 and D_b = 0 as Dirichlet does, and the sine profile is odd about
    every boundary point, so D_b = 0 is also what CD2 would give there."""
    shape = {1: (40,), 2: (17, 23), 3: (9, 11, 13)}[ndim]
    h, a = 0.2, 0.8
    modes = {1: (3,), 2: (2, 5), 3: (1, 3, 4)}[ndim]
    psi = np.ones(shape, dtype=complex)
    lam = 0.0
    for d in range(ndim):
        n = shape[ndim - 1 - d]  # shape is (.., Ny, Nx); axis d counts from x
        m = modes[d]
        i = np.arange(n)
        prof = np.sin(math.pi * m * i / (n - 1))
        sh = [1] * ndim
        sh[ndim - 1 - d] = n
        psi = psi * prof.reshape(sh)
        lam += _lam(math.pi * m / (n - 1), order) / h ** 2
    psi = psi * (0.3 + 0.4j)
    dt = 0.7 * oracle.dt_max(ndim, order, h, a)
    nsteps = 20
    out = oracle.rk4(psi, h, a, 0.0, dt, nsteps, order=order, bc=bc)
    expect = R4(1j * a * dt * lam) ** nsteps * psi
    assert np.max(np.abs(out - expect)) < 1e-13


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("order", [2, 4])
def test_dispersion_planewave_msd(ndim, order):
    """A plane wave has constant modulus, so MSD (Eq. msd / Eq. BCMSDlap) is
    exact for it, and psi^n = R(i a k lambda)^n psi^0 at every point."""
    shape = {1: (31,), 2: (12, 15), 3: (8, 9, 10)}[ndim]
    h, a = 0.25, 1.3
    kap = (0.7, -1.1, 0.5)[:ndim]
    psi = np.ones(shape, dtype=complex)
    lam = 0.0
    for d in range(ndim):
        n = shape[ndim - 1 - d]
        x = np.arange(n) * h
        sh = [1] * ndim
        sh[ndim - 1 - d] = n
        psi = psi * np.exp(1j * kap[d] * x).reshape(sh)
        lam += _lam(kap[d] * h, order) / h ** 2
    dt = 0.8 * oracle.dt_max(ndim, order, h, a)
    nsteps = 25
    out = oracle.rk4(psi, h, a, 0.0, dt, nsteps, order=order, bc="msd")
    expect = R4(1j * a * dt * lam) ** nsteps * psi
    assert np.max(np.abs(out - expect)) < 1e-13


# ---------------------------------------------------------------- Laplacian stencils

def _poly_field(shape, h, degree, seed):
    """Random real polynomial of total degree <= degree on the grid, and its
    exact Laplacian (by differentiating the coefficient array)."""
    from numpy.polynomial import polynomial as P
    ndim = len(shape)
    g = np.random.default_rng(seed)
    c = np.zeros((degree + 1,) * 3)
    for i in range(degree + 1):
        for j in range(degree + 1 - i):
            for k in range(degree + 1 - i - j):
                if (ndim < 2 and j) or (ndim < 3 and k):
                    continue
                c[i, j, k] = g.uniform(-1, 1)
    axes = [np.arange(n) * h - 0.5 for n in reversed(shape)] + [np.zeros(1)] * (3 - ndim)
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    val = P.polyval3d(X, Y, Z, c)
    lap = sum(P.polyval3d(X, Y, Z, P.polyder(c, 2, axis=ax)) for ax in range(3))
    return val.reshape(shape), lap.reshape(shape)


def _deep_interior(shape, w=2):
    return tuple(slice(w, n - w) for n in shape)


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("order,exact_deg", [(2, 3), (4, 5)])
def test_laplacian_polynomial_exactness(ndim, order, exact_deg):
    """CD2 is exact on polynomials of degree <= 3, 2SHOC on degree <= 5 (its
    h^2 mixed terms cancel), and neither on one degree more."""
    shape = {1: (21,), 2: (11, 12), 3: (9, 8, 10)}[ndim]
    h = 0.1
    sl = _deep_interior(shape)
    for deg, exact in ((exact_deg, True), (exact_deg + 1, False)):
        u, lap = _poly_field(shape, h, deg, seed=10 * ndim + deg)
        L = oracle.laplacian(u + 0j, h, order=order)
        err = np.max(np.abs(L[sl] - lap[sl]))
        if exact:
            assert err < 1e-9
        else:
            assert err > 1e-6


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_2shoc_equals_wide_fourth_order_stencil(ndim):
    """In the interior, 2SHOC equals the wide cross stencil
    sum_d (-u_{+-2}/12 + 4/3 u_{+-1} - 5/2 u) / h^2, an independent formula."""
    shape = {1: (30,), 2: (14, 13), 3: (9, 10, 11)}[ndim]
    h = 0.37
    u = wl.random_field(shape, 90 + ndim)
    L = oracle.laplacian(u, h, order=4)
    wide = np.zeros_like(u)
    sl = _deep_interior(shape)
    for ax in range(ndim):
        def sh(k):
            idx = list(sl)
            s = idx[ax]
            idx[ax] = slice(s.start + k, s.stop + k)
            return u[tuple(idx)]
        wide[sl] += (-(sh(2) + sh(-2)) / 12 + 4.0 / 3.0 * (sh(1) + sh(-1)) - 2.5 * sh(0)) / h ** 2
    assert np.max(np.abs(L[sl] - wide[sl])) < 1e-11 * np.max(np.abs(wide[sl]))


# ---------------------------------------------------------------- boundary forms

@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("bc", ["dirichlet", "msd"])
def test_stationary_state_is_fixed_point(ndim, order, bc):
    """Pick a positive cubic P and V = a Lap(P)/P + s P^2, so psi = e^{i phi} P
    is an exact stationary state.  Both schemes are exact on cubics, and both
    Laplacian forms of the boundary conditions (Eqs. BCDlap / BCMSDlap) return
    the exact Laplacian of a stationary state, so every F is zero and RK4 keeps
    psi fixed.  A wrong sign or factor in any boundary form moves it."""
    shape = {1: (15,), 2: (9, 10), 3: (7, 8, 9)}[ndim]
    h, a, s = 0.15, 0.9, -1.3
    p, lap = _poly_field(shape, h, 3, seed=5 + ndim)
    p = 3.0 + 0.2 * p
    lap = 0.2 * lap
    assert p.min() > 0
    V = a * lap / p + s * p * p
    psi = np.exp(0.4j) * p
    dt = 0.8 * oracle.dt_max(ndim, order, h, a)
    out = oracle.rk4(psi, h, a, s, dt, 10, V=V, order=order, bc=bc)
    assert np.max(np.abs(out - psi)) < 1e-12
    F = oracle.rhs(psi, h, a, s, V=V, order=order, bc=bc)
    assert np.max(np.abs(F)) < 1e-11
    # discriminating: a perturbed potential is not stationary
    out2 = oracle.rk4(psi, h, a, s, dt, 10, V=V + 0.01, order=order, bc=bc)
    assert np.max(np.abs(out2 - psi)) > 1e-4


def _scalar_rk4(y, s, v, dt, n):
    """n textbook RK4 steps of the scalar ODE psi' = i (s|psi|^2 - v) psi
    (numpy-broadcast over y and v)."""
    f = lambda z: 1j * (s * np.abs(z) ** 2 - v) * z
    for _ in range(n):
        k1 = f(y); k2 = f(y + dt / 2 * k1); k3 = f(y + dt / 2 * k2); k4 = f(y + dt * k3)
        y = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("bc", ["msd", "l0"])
def test_uniform_field_msd_follows_scalar_rk4(ndim, order, bc):
    """A uniform field under MSD or L0 with uniform V stays uniform; each point
    follows the scalar RK4 recurrence of psi' = i (s|psi|^2 - V) psi.  For
    2SHOC this needs D_b = 0 at the boundary: the Dirichlet form
    -(1/a) N_b psi_b is not zero here and would bend the first interior
    layer."""
    shape = {1: (12,), 2: (7, 9), 3: (5, 6, 7)}[ndim]
    h, a, s, v = 0.2, 1.0, 0.8, 0.35
    psi0 = 0.9 - 0.5j
    V = np.full(shape, v)
    dt = 0.01
    out = oracle.rk4(np.full(shape, psi0), h, a, s, dt, 30, V=V, order=order, bc=bc)
    y = _scalar_rk4(psi0, s, v, dt, 30)
    assert np.max(np.abs(out - y)) < 1e-13


def _boundary_mask(shape):
    m = np.zeros(shape, dtype=bool)
    for ax in range(len(shape)):
        idx = [slice(None)] * len(shape)
        idx[ax] = 0
        m[tuple(idx)] = True
        idx[ax] = -1
        m[tuple(idx)] = True
    return m


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("order", [2, 4])
def test_l0_boundary_points_follow_their_own_scalar_rk4(ndim, order):
    """Under L0 (Eq. BCL0dt) the time derivative of a boundary point depends
    on that point alone, so for any interior field and any potential every
    boundary point follows the scalar RK4 recurrence with its own V_b.
    Dirichlet (frozen) and MSD (coupled to the inward neighbour) both fail
    this, which the test checks too."""
    shape = {1: (14,), 2: (8, 11), 3: (6, 7, 9)}[ndim]
    h, a, s = 0.3, 0.8, -1.1
    u = 1.5 + 0.4 * wl.random_field(shape, 21 + ndim, smooth=1.0)  # |u| > 0 keeps MSD finite
    V = 0.5 * wl.random_field(shape, 21 + ndim, stream=1).real
    dt, n = 0.4 * oracle.dt_max(ndim, order, h, a), 12
    b = _boundary_mask(shape)
    expect = _scalar_rk4(u[b], s, V[b], dt, n)
    out = oracle.rk4(u, h, a, s, dt, n, V=V, order=order, bc="l0")
    assert np.max(np.abs(out[b] - expect)) < 1e-13
    assert np.max(np.abs(out[~b] - u[~b])) > 1e-3  # the interior does move
    for other in ("dirichlet", "msd"):
        o = oracle.rk4(u, h, a, s, dt, n, V=V, order=order, bc=other)
        assert np.max(np.abs(o[b] - expect)) > 1e-4


def test_l0_2shoc_1d_equals_wide_stencil_on_odd_reflection():
    """1D 2SHOC with L0 (D_b = 0, Eq. BCL0lap): extending the field by odd
    reflection about the boundary point, u_{-k} = 2u_0 - u_k, makes the CD2
    value at the boundary exactly zero, so the L0 Laplacian at every interior
    point equals the interior 2SHOC of the extended field, which is the wide
    fourth-order stencil (-u_{+-2}/12 + 4/3 u_{+-1} - 5/2 u)/h^2."""
    n, h = 17, 0.37
    u = wl.random_field((n,), 31)
    L = oracle.laplacian(u, h, a=0.9, s=0.4, order=4, bc="l0")
    ext = np.concatenate([2 * u[0] - u[2:0:-1], u, 2 * u[-1] - u[-2:-4:-1]])  # 2 ghost points each side
    i = np.arange(1, n - 1) + 2
    wide = (-(ext[i + 2] + ext[i - 2]) / 12 + 4 / 3 * (ext[i + 1] + ext[i - 1]) - 2.5 * ext[i]) / h ** 2
    assert np.max(np.abs(L[1:-1] - wide)) < 1e-10 * np.max(np.abs(wide))
    # the MSD form of D_b gives a different first interior layer
    Lm = oracle.laplacian(u, h, a=0.9, s=0.4, order=4, bc="msd")
    assert np.max(np.abs(Lm[1:-1] - wide)) > 1e-3


@pytest.mark.parametrize("order", [2, 4])
def test_l0_stationary_dark_soliton(order):
    """The black soliton tanh(x/sqrt(2a)) e^{-it} (Eq. soliton with zero
    speed, s = -1) has a vanishing Laplacian far from its core, where its
    boundary values obey Eq. BCL0dt up to e^{-2L/sqrt(2a)}.  With L0 the
    error after t = 1 is the discretisation error, falling as h^2 (CD2) or
    h^4 (2SHOC); Dirichlet freezes the rotating boundary values and does far
    worse."""
    a, s, T = 1.0, -1.0, 1.0

    def err(h, bc):
        x = np.arange(-30, 30 + h / 2, h)
        ex0 = wl.dark_soliton1d_exact(x, 0.0, a=a, s=s, c=0.0)
        exT = wl.dark_soliton1d_exact(x, T, a=a, s=s, c=0.0)
        dt = 0.8 * oracle.dt_max(1, order, h, a)
        nst = int(math.ceil(T / dt))
        out = oracle.rk4(ex0, h, a, s, T / nst, nst, order=order, bc=bc)
        return np.linalg.norm(out - exT) / np.linalg.norm(exT)

    e1, e2 = err(0.2, "l0"), err(0.1, "l0")
    assert math.log2(e1 / e2) == pytest.approx(order, abs=0.15)
    assert err(0.2, "dirichlet") > 10 * e1


def test_dirichlet_boundary_frozen_and_rhs_zero():
    u = wl.random_field((9, 11), 7)
    F = oracle.rhs(u, 0.3, 1.0, 1.0, order=4, bc="dirichlet")
    assert np.all(F[0, :] == 0) and np.all(F[-1, :] == 0)
    assert np.all(F[:, 0] == 0) and np.all(F[:, -1] == 0)
    out = oracle.rk4(u, 0.3, 1.0, 1.0, 1e-3, 5, order=2, bc="dirichlet")
    assert np.array_equal(out[0, :], u[0, :]) and np.array_equal(out[:, -1], u[:, -1])


# ---------------------------------------------------------------- exact solutions, orders

@pytest.mark.parametrize("order,expected", [(2, 1.03e-2), (4, 4.61e-5)])
def test_bright_soliton_c1(order, expected):
    """The 1024-point bright soliton after 1000 steps at 0.8 of the bound:
    the error against the exact solution is the discretisation error."""
    p = wl.soliton1d(order=order)
    dt = 0.8 * oracle.dt_max(1, order, p.h, p.a)
    out = oracle.rk4(p.psi0, p.h, p.a, p.s, dt, 1000, order=order, bc="dirichlet")
    ex = wl.soliton1d_exact(p.meta["x"], 1000 * dt)
    err = np.linalg.norm(out - ex) / np.linalg.norm(ex)
    assert err == pytest.approx(expected, rel=0.05)


def _soliton_err(order, h, T, kind):
    a = 1.0
    if kind == "bright":
        s = 1.0
        x = np.arange(-20, 20 + h / 2, h)
        ex0, exT = wl.soliton1d_exact(x, 0.0), wl.soliton1d_exact(x, T)
        bc = "dirichlet"
    else:
        s = -1.0
        x = np.arange(-40, 40 + h / 2, h)
        ex0, exT = wl.dark_soliton1d_exact(x, 0.0), wl.dark_soliton1d_exact(x, T)
        bc = "msd"
    dt = 0.8 * oracle.dt_max(1, order, h, a)
    n = int(math.ceil(T / dt))
    out = oracle.rk4(ex0, h, a, s, T / n, n, order=order, bc=bc)
    return np.linalg.norm(out - exT) / np.linalg.norm(exT)


@pytest.mark.parametrize("kind", ["bright", "dark"])
@pytest.mark.parametrize("order", [2, 4])
def test_spatial_convergence_order(kind, order):
    """dt proportional to h^2: the error falls as h^2 (CD2) or h^4 (2SHOC).
    The dark soliton (Eq. soliton) runs with MSD boundaries."""
    e1 = _soliton_err(order, 0.2, 1.0, kind)
    e2 = _soliton_err(order, 0.1, 1.0, kind)
    rate = math.log2(e1 / e2)
    assert rate == pytest.approx(order, abs=0.15)


def test_time_convergence_order():
    """Linear sine mode: RK4 error against the exact semi-discrete solution
    e^{i a lambda t} falls as k^4."""
    n, h, a, m = 32, 0.5, 1.0, 3
    i = np.arange(n)
    psi = np.sin(math.pi * m * i / (n - 1)) + 0j
    lam = _lam(math.pi * m / (n - 1), 2) / h ** 2
    T = 2.0
    errs = []
    for nst in (20, 40):
        out = oracle.rk4(psi, h, a, 0.0, T / nst, nst, order=2, bc="dirichlet")
        errs.append(np.max(np.abs(out - np.exp(1j * a * lam * T) * psi)))
    assert math.log2(errs[0] / errs[1]) == pytest.approx(4.0, abs=0.1)


def test_stability_threshold_highest_mode():
    """The highest Dirichlet sine mode grows iff k |lambda_max| > 2 sqrt 2."""
    n, h, a = 24, 0.2, 1.0
    m = n - 2
    i = np.arange(n)
    psi = np.sin(math.pi * m * i / (n - 1)) + 0j
    lam = abs(_lam(math.pi * m / (n - 1), 2)) / h ** 2
    kcrit = 2 * math.sqrt(2) / (a * lam)
    grow = oracle.rk4(psi, h, a, 0.0, 1.02 * kcrit, 400, order=2, bc="dirichlet")
    keep = oracle.rk4(psi, h, a, 0.0, 0.98 * kcrit, 400, order=2, bc="dirichlet")
    assert np.max(np.abs(grow)) > 2.0
    assert np.max(np.abs(keep)) <= 1.0 + 1e-12
    assert kcrit >= oracle.dt_max(1, 2, h, a)


# ---------------------------------------------------------------- invariants

def test_mass_energy_soliton_closed_forms():
    """Continuum values for the bright soliton: M = 4 sqrt(ca)/s and
    E = -(4/3) c^{3/2} sqrt(a)/s.  The discrete mass is spectrally accurate;
    the discrete energy converges at order 2 (CD2) and 4 (2SHOC)."""
    M_ex, E_ex = 4.0, -4.0 / 3.0
    for order in (2, 4):
        errs = []
        for n in (257, 513):
            L = 40.0
            h = L / (n - 1)
            x = -L / 2 + np.arange(n) * h
            psi = wl.soliton1d_exact(x, 0.0)
            M, E = oracle.mass_energy(psi, h, 1.0, 1.0, order=order)
            assert M == pytest.approx(M_ex, rel=1e-10)
            errs.append(abs(E - E_ex))
        assert math.log2(errs[0] / errs[1]) == pytest.approx(order, abs=0.15)


def test_energy_kinetic_summation_by_parts():
    """For a field that vanishes on the boundary, -sum_int conj(u) CD2(u)
    equals the forward-difference form sum |u_{i+1} - u_i|^2 / h^2."""
    u = wl.random_field((12, 14), 3, smooth=2.0)
    u[0, :] = u[-1, :] = 0
    u[:, 0] = u[:, -1] = 0
    h = 0.3
    M, E = oracle.mass_energy(u, h, 1.0, 0.0, order=2)
    kin = (np.sum(np.abs(np.diff(u, axis=0)) ** 2) + np.sum(np.abs(np.diff(u, axis=1)) ** 2))
    assert E == pytest.approx(kin, rel=1e-12)  # h^2 * kin / h^2
    assert M == pytest.approx(h * h * np.sum(np.abs(u) ** 2), rel=1e-14)


@pytest.mark.parametrize("order,tol_m,tol_e", [(2, 1e-10, 1e-9), (4, 1e-10, 1e-9)])
def test_conservation_soliton(order, tol_m, tol_e):
    """Mass and (scheme-consistent) energy are conserved up to the small RK4
    drift for a localised field with zero Dirichlet boundaries."""
    p = wl.soliton1d(order=order)
    dt = 0.8 * oracle.dt_max(1, order, p.h, p.a)
    M0, E0 = oracle.mass_energy(p.psi0, p.h, p.a, p.s, order=order)
    out = oracle.rk4(p.psi0, p.h, p.a, p.s, dt, 1000, order=order)
    M1, E1 = oracle.mass_energy(out, p.h, p.a, p.s, order=order)
    assert abs(M1 - M0) / M0 < tol_m
    assert abs(E1 - E0) / abs(E0) < tol_e


def _packet_in_trap(dim):
    """A Gaussian wave packet with momentum, off-centre in a harmonic trap,
    small at the (zero Dirichlet) edges of the box."""
    if dim == 1:
        h = 0.1
        x = -20 + np.arange(401) * h
        psi = 0.8 * np.exp(-(x + 4) ** 2 / (2 * 1.5 ** 2)) * np.exp(1j * x)
        V = 0.1 * x ** 2
    else:
        h = 0.25
        x = -10 + np.arange(81) * h
        Y, X = np.meshgrid(x, x, indexing="ij")
        psi = 0.8 * np.exp(-((X + 3) ** 2 + (Y - 1) ** 2) / (2 * 1.2 ** 2)) * np.exp(1j * (0.8 * X + 0.3 * Y))
        V = 0.5 * (0.25 * X ** 2 + 0.15 * Y ** 2)
    return psi, V, h


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("order", [2, 4])
def test_energy_conserved_while_packet_moves_in_static_potential(dim, order):
    """The Hamiltonian of i psi_t = -a Lap psi + V psi - s|psi|^2 psi includes
    +V|psi|^2 with a static V, so E stays constant while the packet rolls
    down the trap and its potential energy h^d sum V|psi|^2 changes by a few
    percent of E.  A wrong sign or factor of the potential term in E would
    make E change by a multiple of that (the potential energy is computed
    here independently of the oracle's energy)."""
    psi, V, h = _packet_in_trap(dim)
    a, s = 1.0, -1.0
    dt = 0.5 * oracle.dt_max(dim, order, h, a)
    nst = int(2.0 / dt)
    M0, E0 = oracle.mass_energy(psi, h, a, s, V=V, order=order)
    out = oracle.rk4(psi, h, a, s, dt, nst, V=V, order=order)
    M1, E1 = oracle.mass_energy(out, h, a, s, V=V, order=order)
    pot0 = h ** dim * np.sum(V * np.abs(psi) ** 2)
    pot1 = h ** dim * np.sum(V * np.abs(out) ** 2)
    assert abs(pot1 - pot0) / abs(E0) > 1e-2  # the packet really moved in V
    assert abs(M1 - M0) / M0 < 1e-6
    assert abs(E1 - E0) / abs(E0) < 1e-6


@pytest.mark.parametrize("shape,order,bc", [((40,), 2, "dirichlet"), ((40,), 4, "msd"),
                                            ((12, 14), 4, "dirichlet"), ((12, 14), 2, "l0"),
                                            ((6, 7, 8), 4, "msd"), ((6, 7, 8), 2, "dirichlet")])
def test_energy_shift_by_constant_potential(shape, order, bc):
    """A constant potential V = c only shifts the Hamiltonian by c times the
    mass: E(V = c) - E(V = 0) = c M.  (For 2SHOC with Dirichlet or MSD the
    boundary D depends on V through N_b; a constant V cancels in N_q - N_b
    for MSD but not for Dirichlet, so Dirichlet + 2SHOC is checked with a
    field that vanishes on the boundary.)"""
    u = 1.2 + 0.4 * wl.random_field(shape, 11, smooth=2.0)
    if bc == "dirichlet":
        for ax in range(len(shape)):
            idx = [slice(None)] * len(shape)
            idx[ax] = 0
            u[tuple(idx)] = 0
            idx[ax] = -1
            u[tuple(idx)] = 0
    h, a, s, c = 0.3, 0.7, -1.0, 0.625
    M0, E0 = oracle.mass_energy(u, h, a, s, V=None, order=order, bc=bc)
    Mc, Ec = oracle.mass_energy(u, h, a, s, V=np.full(shape, c), order=order, bc=bc)
    assert Mc == M0
    assert Ec - E0 == pytest.approx(c * M0, rel=1e-12, abs=1e-12 * abs(E0))


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.rk4(np.zeros(2, complex), 0.1, 1.0, 1.0, 1e-3, 1)
    with pytest.raises(ValueError):
        oracle.rk4(np.zeros(8, complex), -0.1, 1.0, 1.0, 1e-3, 1)
    with pytest.raises(ValueError):
        oracle.rk4(np.zeros(8, complex), 0.1, 1.0, 1.0, 1e-3, 1, order=3)
    lib = oracle._load()
    u = np.zeros(16)
    n = (ctypes.c_long * 3)(8, 1, 1)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.orc_rk4(1, n, 0.1, 1.0, 1.0, None, 2, 3, 1e-3, 1, u.ctypes.data_as(dp)) != 0  # bc 3 unknown
