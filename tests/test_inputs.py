"""Pins of the input generators that carry arithmetic of their own: the
numerically exact dark-vortex profile (Eq. exmp2Dvort) and the inputs built
from it (Eq. 3dvr1).

The profile g solves a (g'' + g'/r - m^2 g/r^2) + (1 - g^2) g = 0, g(0) = 0,
g(inf) = 1.  The checks use facts derived from that equation, not the
solver's own discretisation: the residual under an independent
fourth-order difference formula, the near-core series, the far-field
expansion, grid convergence, and (through the CPU oracle) that a vortex with
this core stays put far better than one with the tanh core.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1203_1263_amd import workloads as wl


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_profile_solves_the_radial_equation(a):
    """Residual of the continuous equation under independent fourth-order
    difference formulas, away from the singular point r = 0: small, and
    falling as dr^2 (the solver's own order)."""
    res = []
    for dr in (0.01, 0.005):
        r, g = wl.vortex_profile(1, a, rmax=30.0, dr=dr)
        i = np.arange(4, len(r) - 4)
        g1 = (-g[i + 2] + 8 * g[i + 1] - 8 * g[i - 1] + g[i - 2]) / (12 * dr)
        g2 = (-g[i + 2] + 16 * g[i + 1] - 30 * g[i] + 16 * g[i - 1] - g[i - 2]) / (12 * dr * dr)
        ri = r[i]
        rr = a * (g2 + g1 / ri - g[i] / ri ** 2) + (1 - g[i] ** 2) * g[i]
        res.append(np.max(np.abs(rr[ri > 0.1])))
    assert res[1] < 3e-5
    assert math.log2(res[0] / res[1]) == pytest.approx(2.0, abs=0.2)


def test_profile_near_core_series_and_far_field():
    """Near r = 0: g = c r - (c/(8a)) r^3 + O(r^5) (the r^3 coefficient
    follows from the equation).  Far away: g = 1 - a/(2 r^2) + O(r^-4)."""
    for a in (1.0, 0.5):
        r, g = wl.vortex_profile(1, a, rmax=40.0, dr=0.002)
        k = (r > 0) & (r < 0.3)
        c = np.polyfit(r[k] ** 2, g[k] / r[k], 2)  # g/r = c0 + c2 r^2 + c4 r^4
        assert c[1] == pytest.approx(-c[2] / (8 * a), rel=2e-3)
        for rr in (10.0, 15.0, 20.0):
            j = int(round(rr / 0.002))
            assert abs(g[j] - (1 - a / (2 * rr * rr))) < 3 * a * a / rr ** 4
    # the length scale is sqrt(a): profiles for a and a' agree after r -> r sqrt(a'/a)
    r1, g1 = wl.vortex_profile(1, 1.0, rmax=40.0, dr=0.004)
    r2, g2 = wl.vortex_profile(1, 0.25, rmax=20.0, dr=0.002)
    assert np.max(np.abs(np.interp(r2 * 2.0, r1, g1) - g2)) < 1e-4


def test_profile_grid_convergence():
    r1, g1 = wl.vortex_profile(1, 1.0, dr=0.02)
    r2, g2 = wl.vortex_profile(1, 1.0, dr=0.01)
    r3, g3 = wl.vortex_profile(1, 1.0, dr=0.005)
    e1 = np.max(np.abs(g1 - g3[::4]))
    e2 = np.max(np.abs(g2 - g3[::2]))
    # second order against the dr = 0.005 solution: (0.02^2 - 0.005^2) / (0.01^2 - 0.005^2) = 5
    assert e1 / e2 == pytest.approx(5.0, rel=0.1)


def test_exact_core_vortex_is_nearly_stationary():
    """A single charge-1 vortex on a unit background evolved by the oracle
    (2SHOC, MSD, t = 2): the density of the exact-core vortex changes far
    less than that of the tanh-core one, which is not a stationary state."""
    n, h = 97, 0.4
    x = wl.axis(n, h)
    prof = wl.vortex_profile(1, 1.0)
    dt = 0.5 * oracle.dt_max(2, 4, h, 1.0)
    nst = int(round(2.0 / dt))
    change = {}
    for name, p in (("exact", prof), ("tanh", None)):
        psi = wl.vortex_field(x, x, [(0.0, 0.0)], [1], profile=p, a=1.0)
        out = oracle.rk4(psi, h, 1.0, -1.0, dt, nst, order=4, bc="msd")
        core = np.abs(psi) < 0.99  # where the profile differs from the background
        change[name] = np.max(np.abs(np.abs(out[core]) - np.abs(psi[core])))
    assert change["exact"] < 0.01 * change["tanh"]  # measured 1.8e-4 against 0.24
    assert change["exact"] < 1e-3


def test_paper_ring_input():
    p = wl.ring3d_paper(shape=(24, 28, 28), h=0.5, d=4.0)
    assert p.V is None and p.s == -1.0
    m = np.abs(p.psi0)
    assert m.max() <= 1.0 and m.min() < 0.2  # unit background, a dark core
    assert p.meta["c"] == pytest.approx(wl.ring_velocity(4.0, 1.0))
    # the ring speed law: ln growth with radius, 1/d decay
    assert wl.ring_velocity(8.0, 1.0) < wl.ring_velocity(4.0, 1.0)
    assert wl.ring_velocity(4.0, 0.5) == pytest.approx(0.5 / 4.0 * (math.log(8 * 4.0) - 0.615))


def test_townes_mass_constant():
    """The critical mass used by the batch workload: the 2D ground state of
    R'' + R'/r - R + R^3 = 0 (R'(0) = 0, R -> 0) found by shooting on R(0)
    (too small: R turns back up; too large: R crosses zero), its mass
    2 pi int R^2 r dr against TOWNES_MASS."""
    from scipy.integrate import solve_ivp

    def shoot(r0, rmax=12.0):
        def f(r, y):
            return [y[1], -y[1] / r + y[0] - y[0] ** 3]
        r1 = 1e-6  # series start: R = r0 + (r0 - r0^3) r^2 / 4
        y1 = [r0 + (r0 - r0 ** 3) * r1 * r1 / 4, (r0 - r0 ** 3) * r1 / 2]
        cross = lambda r, y: y[0]
        cross.terminal = True
        turn = lambda r, y: y[1]
        turn.terminal = True
        turn.direction = 1
        sol = solve_ivp(f, (r1, rmax), y1, rtol=1e-12, atol=1e-14, events=(cross, turn), dense_output=True)
        return sol

    lo, hi = 2.0, 2.5
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        sol = shoot(mid)
        if sol.t_events[0].size:  # crossed zero: start too high
            hi = mid
        else:
            lo = mid
    sol = shoot(0.5 * (lo + hi), rmax=8.0)
    r = np.linspace(1e-6, sol.t[-1], 20001)
    R = sol.sol(r)[0]
    mass = 2 * np.pi * np.trapezoid(R * R * r, r)
    assert 2.20 < 0.5 * (lo + hi) < 2.21          # R(0) of the Townes profile
    assert mass == pytest.approx(wl.TOWNES_MASS, rel=2e-4)


def test_batch_focusing_problems_stay_below_half_the_critical_mass():
    """Every focusing problem of the batched workload starts at or below half
    the critical mass TOWNES_MASS * a / s (so none can collapse); the
    defocusing ones keep max |psi|^2 = 1."""
    for p in wl.batch2d():
        mass = p.h * p.h * float(np.sum(np.abs(p.psi0) ** 2))
        if p.s > 0:
            assert mass <= 0.5 * wl.TOWNES_MASS * p.a / p.s * (1 + 1e-12)
        else:
            assert np.max(np.abs(p.psi0) ** 2) == pytest.approx(1.0)
