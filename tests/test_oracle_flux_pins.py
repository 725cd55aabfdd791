"""Pins of the oracle's HLLC edge flux (cfg.flux = 1, adiabatic closure),
against what the flux must do rather than its formula:

* consistency: h(U, U) = f(U).n;
* an isolated contact at rest (density jump, equal pressure, any jump of the
  tangential velocity) is kept exactly: no mass, energy or tangential momentum
  crosses it, where the Rusanov flux of the same states lets mass through;
* a moving contact is upwinded exactly: h = f(U_upwind).n in both directions;
* the flux is continuous along a Galilean boost of a Riemann problem, through
  the points where the contact or an outer wave is at rest;
* supersonic flow: h = f(U_upwind).n;
* conservation between the two elements of an edge: h(U_L, U_R, n) =
  -h(U_R, U_L, -n) to rounding;
* the whole DG solver (order 2, positivity limiter) on Sod's shock tube
  converges to the exact Riemann solution (written here from the textbook's
  exact solver: pressure from the two wave curves by bisection), with smaller
  L1 errors than the Rusanov flux.
A dropped or mis-signed term of the contact speed fails the moving contact,
a wrong star state the continuity (the shock tube does not see every such
mistake: a consistent flux with a different dissipation still converges).
"""
import math

import numpy as np
import pytest

import oracle as O

G = 1.4


def cfg(flux, **kw):
    return O.cfg(closure=2, nvar=4, gamma=G, flux=flux, **kw)


def cons(rho, vx, vy, p):
    return np.array([rho, rho * vx, rho * vy, p / (G - 1) + 0.5 * rho * (vx * vx + vy * vy)])


def phys_flux(U, nx, ny):
    rho, mx, my, E = U
    vx, vy = mx / rho, my / rho
    p = (G - 1) * (E - 0.5 * rho * (vx * vx + vy * vy))
    q = vx * nx + vy * ny
    return np.array([rho * q, mx * q + p * nx, my * q + p * ny, (E + p) * q])


NORMALS = [(1.0, 0.0), (-1.0, 0.0), (0.0, 1.0), (0.0, -1.0)]


@pytest.mark.parametrize("n", NORMALS)
def test_hllc_is_consistent(n):
    rng = np.random.default_rng(1)
    c = cfg(1)
    for _ in range(20):
        U = cons(rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.1, 5))
        h = O.num_flux(c, U, U, *n)
        f = phys_flux(U, *n)
        assert np.allclose(h, f, rtol=1e-14, atol=1e-14 * np.abs(f).max()), (h, f)


@pytest.mark.parametrize("n", NORMALS)
def test_contact_at_rest_is_kept_exactly(n):
    nx, ny = n
    # density jump, equal pressure, no normal velocity, a jump of the
    # tangential velocity (a shear layer on the contact)
    t = (-ny, nx)
    UL = cons(1.0, 0.3 * t[0], 0.3 * t[1], 2.5)
    UR = cons(0.125, -0.7 * t[0], -0.7 * t[1], 2.5)
    h = O.num_flux(cfg(1), UL, UR, nx, ny)
    want = np.array([0.0, 2.5 * nx, 2.5 * ny, 0.0])
    assert np.allclose(h, want, atol=1e-14), h
    # the Rusanov flux of the same states lets mass through
    r = O.num_flux(cfg(0), UL, UR, nx, ny)
    assert abs(r[0]) > 0.1


@pytest.mark.parametrize("n", NORMALS)
@pytest.mark.parametrize("u", [0.4, -0.4])
def test_moving_contact_is_upwinded(n, u):
    nx, ny = n
    UL = cons(1.0, u * nx + 0.2 * ny, u * ny - 0.2 * nx, 1.0)
    UR = cons(0.3, u * nx - 0.5 * ny, u * ny + 0.5 * nx, 1.0)
    h = O.num_flux(cfg(1), UL, UR, nx, ny)
    want = phys_flux(UL if u > 0 else UR, nx, ny)
    assert np.allclose(h, want, rtol=1e-13, atol=1e-13), (h, want)


@pytest.mark.parametrize("n", NORMALS)
def test_supersonic_flow_is_upwinded(n):
    nx, ny = n
    for q in (3.0, -3.0):  # |q| above both sound speeds
        UL = cons(1.0, q * nx, q * ny, 1.0)
        UR = cons(0.5, q * nx + 0.3 * ny, q * ny - 0.3 * nx, 0.6)
        h = O.num_flux(cfg(1), UL, UR, nx, ny)
        want = phys_flux(UL if q > 0 else UR, nx, ny)
        assert np.allclose(h, want, rtol=1e-14, atol=1e-14), (q, h, want)


def test_flux_is_conservative_between_the_two_elements():
    rng = np.random.default_rng(2)
    c = cfg(1)
    for _ in range(50):
        UL = cons(rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.1, 5))
        UR = cons(rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.1, 5))
        for nx, ny in NORMALS:
            a = O.num_flux(c, UL, UR, nx, ny)
            b = O.num_flux(c, UR, UL, -nx, -ny)
            assert np.allclose(a, -b, rtol=1e-12, atol=1e-12 * np.abs(a).max()), (a, b)


@pytest.mark.parametrize("n", NORMALS)
def test_flux_is_continuous_under_a_galilean_boost(n):
    """Adding a velocity w along n to both states moves every wave speed,
    the contact's included, by w; the HLLC flux is continuous in the states,
    so along w it has no jump where the contact speed, or an outer wave
    speed, passes through zero (the star states meet the jump conditions
    across the contact)."""
    nx, ny = n
    c = cfg(1)
    ws = np.linspace(-2.5, 2.5, 25001)
    dw = ws[1] - ws[0]
    H = np.array([O.num_flux(c, cons(1.0, w * nx + 0.3 * ny, w * ny - 0.3 * nx, 1.0),
                             cons(0.3, (w - 0.4) * nx - 0.2 * ny, (w - 0.4) * ny + 0.2 * nx, 0.25), nx, ny)
                  for w in ws])
    jump = np.abs(np.diff(H, axis=0)).max(axis=0)
    assert (jump < 200 * dw).all(), jump


def sod_exact_density(x, t, rl=1.0, pl=1.0, rr=0.125, pr=0.1, x0=0.5):
    """Exact solution of the Riemann problem with both states at rest: the
    star pressure solves f_L(p) + f_R(p) = 0 (shock or rarefaction wave
    curves), found by bisection; then the rarefaction fan, the contact and the
    shock."""
    cl, cr = math.sqrt(G * pl / rl), math.sqrt(G * pr / rr)

    def f(p, rk, pk, ck):
        if p > pk:
            a, b = 2 / ((G + 1) * rk), (G - 1) / (G + 1) * pk
            return (p - pk) * math.sqrt(a / (p + b))
        return 2 * ck / (G - 1) * ((p / pk) ** ((G - 1) / (2 * G)) - 1)

    lo, hi = 1e-10, 10.0
    for _ in range(200):
        m = 0.5 * (lo + hi)
        lo, hi = (lo, m) if f(m, rl, pl, cl) + f(m, rr, pr, cr) > 0 else (m, hi)
    ps = 0.5 * (lo + hi)
    us = 0.5 * (f(ps, rr, pr, cr) - f(ps, rl, pl, cl))
    rsl = rl * (ps / pl) ** (1 / G)
    g1 = (G - 1) / (G + 1)
    rsr = rr * (ps / pr + g1) / (g1 * ps / pr + 1)
    shock = cr * math.sqrt((G + 1) / (2 * G) * ps / pr + (G - 1) / (2 * G))
    tail = us - cl * (ps / pl) ** ((G - 1) / (2 * G))
    s = (x - x0) / t
    out = np.where(s < -cl, rl, 0.0)
    fan = (s >= -cl) & (s < tail)
    uf = 2 / (G + 1) * (cl + s)
    out = np.where(fan, rl * (np.clip(cl - (G - 1) / 2 * uf, 0, None) / cl) ** (2 / (G - 1)), out)
    out = np.where((s >= tail) & (s < us), rsl, out)
    out = np.where((s >= us) & (s < shock), rsr, out)
    out = np.where(s >= shock, rr, out)
    return out


def sod_error(nx, flux, T=0.2):
    c = O.cfg(n=2, nvar=4, nx=nx, ny=2, x0=0.0, x1=1.0, y0=0.0, y1=2.0 / nx, closure=2, gamma=G, bc=2,
              cfl=0.2, flux=flux, positivity=1)
    x, _ = O.nodes(c)
    x = x.reshape(2 * nx, 4)
    rho = np.where(x < 0.5, 1.0, 0.125)
    p = np.where(x < 0.5, 1.0, 0.1)
    u = O.project(c, np.stack([rho, 0 * rho, 0 * rho, p]))
    u0 = u.copy()
    t = 0.0
    while t < T - 1e-12:
        dt = min(O.dt(c, u), T - t)
        u, _ = O.step_limited(c, u, t, dt, u0, math.inf)
        t += dt
    means = u[0, 0, :].reshape(2, nx)[0]
    xs = (np.arange(nx)[:, None] + (np.arange(64)[None, :] + 0.5) / 64) / nx
    ex = sod_exact_density(xs.ravel(), T).reshape(nx, 64).mean(1)
    return float(np.mean(np.abs(means - ex)))


def test_sod_shock_tube_converges_to_the_exact_solution():
    e50, e100 = sod_error(50, 1), sod_error(100, 1)
    r100 = sod_error(100, 0)
    print(f"[sod] HLLC L1 density error {e50:.3e} (50), {e100:.3e} (100); Rusanov {r100:.3e} (100)")
    assert e100 < 0.75 * e50
    assert e100 < 7e-3
    assert e100 < r100
