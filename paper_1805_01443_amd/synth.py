"""Seeded synthetic initial conditions.

This module only evaluates the problem set-ups (initial primitive fields at
caller-supplied coordinates) and draws seeded random numbers.  It holds none of
the discontinuous Galerkin arithmetic: no quadrature, no basis, no fluxes.  Both
the HIP path (through ``dg_init``) and the CPU oracle receive the arrays it
returns, so the two sides see identical input bits.

Set-ups:

* ``periodic_wave``   density wave rho = 1 + 0.2 sin(2 pi (x + y)) carried by a
  uniform velocity (1, 1) on the periodic unit square (isothermal, c_s = 1).
* ``entropy_wave``    the same wave for the adiabatic equations with p = 1; it is
  an exact solution, translated with velocity (1, 1).
* ``disc``            the planet-disc set-up: surface density
  Sigma0 * max(r, r_c)^(-1/2), locally isothermal sound speed
  c_s^2 = h^2 GM / max(r, r_c) and the azimuthal velocity of rotational
  equilibrium v_phi^2 = r dPhi*/dr + (r / Sigma) d(c_s^2 Sigma)/dr (Sec. 5.1 of
  the paper, with the stellar potential read as a harmonic core inside r_c and
  Keplerian outside, the reading of its Omega^2(r) definition).
* ``disc_ring``       the adiabatic disc (gamma = 1.4, p = c_s^2 Sigma) with an
  axisymmetric Gaussian over-pressure ring p *= 1 + 4 exp(-(r-r_ring)^2/(2 s^2)).
* ``apply_jump``      that state with density and pressure multiplied by a seeded
  factor inside a seeded radius (``ring_jump``): a discontinuity through the
  middle of elements, for the troubled-cell indicators.

Random numbers come from SplitMix64 (Steele, Lea & Flood 2014): the 64-bit
state is ``seed * 0x9E3779B97F4A7C15 + (index + 1) * 0x9E3779B97F4A7C15`` and one
output is the standard mix of that state; the top 53 bits give a double in
[0, 1).
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, index) -> np.ndarray:
    """One SplitMix64 output per (seed, index) pair, as uint64."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) * _GOLDEN + (idx + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, index) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of SplitMix64."""
    z = splitmix64(seed, index)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------------------
# set-ups; every function takes coordinate arrays of any (equal) shape and
# returns a tuple of primitive arrays of that shape.
# ---------------------------------------------------------------------------

def periodic_wave(x, y):
    """(rho, vx, vy): rho = 1 + 0.2 sin(2 pi (x + y)), v = (1, 1)."""
    rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * (x + y))
    return rho, np.ones_like(rho), np.ones_like(rho)


def entropy_wave(x, y, t=0.0):
    """(rho, vx, vy, p) of the adiabatic entropy wave at time t."""
    rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * (x + y - 2.0 * t))
    one = np.ones_like(rho)
    return rho, one, one.copy(), one.copy()


def _disc_fields(x, y, gm, h, r_core, sigma0):
    r = np.sqrt(x * x + y * y)
    rr = np.maximum(r, r_core)
    sigma = sigma0 / np.sqrt(rr)
    cs2 = h * h * gm / rr
    # angular velocity of rotational equilibrium
    inner = r < r_core
    om2 = np.where(inner, gm / r_core ** 3, gm * (1.0 - 1.5 * h * h) / np.maximum(r, 1e-300) ** 3)
    om = np.sqrt(om2)
    vx = -om * y
    vy = om * x
    return sigma, vx, vy, cs2, r


def disc_sigma0(seed):
    """Sigma0 ~ U[0.5, 2] drawn from the seed (index 2**62 is reserved for it)."""
    return 0.5 + 1.5 * float(uniform01(seed, np.uint64(1) << np.uint64(62)))


def disc(x, y, gm=1.0, h=0.05, r_core=0.4, sigma0=1.0, noise_seed=None,
         noise_amp=1e-4, node_ids=None):
    """(rho, vx, vy) of the locally isothermal disc in rotational equilibrium.

    With ``noise_seed`` the density gets rho *= 1 + amp * xi, xi ~ U[-1, 1)
    drawn per node from SplitMix64(noise_seed, node id); ``node_ids`` are the
    global node indices (defaults to the flat index of ``x``).
    """
    sigma, vx, vy, _, _ = _disc_fields(x, y, gm, h, r_core, sigma0)
    if noise_seed is not None:
        ids = np.arange(np.size(x), dtype=np.uint64).reshape(np.shape(x)) if node_ids is None else node_ids
        xi = 2.0 * uniform01(noise_seed, ids) - 1.0
        sigma = sigma * (1.0 + noise_amp * xi)
    return sigma, vx, vy


def disc_ring(x, y, gm=1.0, h=0.05, r_core=0.4, sigma0=1.0, r_ring=1.6,
              width=0.05, peak=5.0):
    """(rho, vx, vy, p) of the adiabatic disc plus an over-pressure ring."""
    sigma, vx, vy, cs2, r = _disc_fields(x, y, gm, h, r_core, sigma0)
    p = cs2 * sigma * (1.0 + (peak - 1.0) * np.exp(-((r - r_ring) ** 2) / (2.0 * width * width)))
    return sigma, vx, vy, p


def isentropic_vortex(x, y, t=0.0, beta=5.0, gamma=1.4, box=10.0, xc=5.0, yc=5.0):
    """(rho, vx, vy, p) of the isentropic vortex of Sec. 4.1 on the periodic
    box [0, box]^2, advected by the free stream (1, 1): the exact solution at
    time t is the initial vortex centred at (xc + t, yc + t) (nearest periodic
    image)."""
    dx = np.mod(x - xc - t + 0.5 * box, box) - 0.5 * box
    dy = np.mod(y - yc - t + 0.5 * box, box) - 0.5 * box
    r2 = dx * dx + dy * dy
    e = np.exp(1.0 - r2)
    rho = (1.0 - (gamma - 1.0) * beta ** 2 / (8.0 * gamma * np.pi ** 2) * e) ** (1.0 / (gamma - 1.0))
    g = beta / (2.0 * np.pi) * np.sqrt(e)
    return rho, 1.0 - g * dy, 1.0 + g * dx, rho ** gamma


def gresho(x, y, xc=0.5, yc=0.5):
    """(rho, vx, vy, p) of the Gresho vortex of Sec. 4.2: rho = 1, v_phi =
    5r, 2 - 5r, 0 on r < 0.2, 0.2 <= r < 0.4, r >= 0.4, and the pressure that
    balances it."""
    dx, dy = x - xc, y - yc
    r = np.sqrt(dx * dx + dy * dy)
    inner, mid = r < 0.2, (r >= 0.2) & (r < 0.4)
    vphi = np.where(inner, 5.0 * r, np.where(mid, 2.0 - 5.0 * r, 0.0))
    rs = np.maximum(r, 1e-300)
    p = np.where(inner, 5.0 + 12.5 * r * r,
                 np.where(mid, 9.0 - 4.0 * np.log(0.2) + 12.5 * r * r - 20.0 * r + 4.0 * np.log(rs),
                          3.0 + 4.0 * np.log(2.0)))
    return np.ones_like(r), -vphi * dy / rs, vphi * dx / rs, p


def gresho_vorticity(x, y, xc=0.5, yc=0.5):
    """Exact vorticity of the Gresho vortex: 10, 2/r - 10, 0."""
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    return np.where(r < 0.2, 10.0, np.where(r < 0.4, 2.0 / np.maximum(r, 1e-300) - 10.0, 0.0))


def paper_disc(x, y, gm=1.0, sigma0=1.0, p0=2.5e-3, r_in=0.4, r_ex=1.75, h=0.05, rp=1.0):
    """(Sigma, vx, vy, p) of the adiabatic disc of Sec. 5.1: Sigma = Sigma0/(1+f),
    p = p0/(1+f), f = exp((r - r_ex)/(r_p h)); rotational equilibrium
    v_phi^2 = r^2 Omega^2 - r c_iso^2 f / (r_p h (1+f)), c_iso^2 = p0/Sigma0,
    with Omega^2 = GM/r_in^3 inside r_in (solid rotation) and GM/r^3 outside
    (the printed formula's leading "Omega^2" read as r^2 Omega^2)."""
    r = np.sqrt(x * x + y * y)
    f = np.exp((r - r_ex) / (rp * h))
    sigma = sigma0 / (1.0 + f)
    p = p0 / (1.0 + f)
    om2 = np.where(r <= r_in, gm / r_in ** 3, gm / np.maximum(r, 1e-300) ** 3)
    c2 = p0 / sigma0
    vphi2 = r * r * om2 - r * c2 * f / (rp * h * (1.0 + f))
    vphi = np.sqrt(np.maximum(vphi2, 0.0))
    rs = np.maximum(r, 1e-300)
    return sigma, -vphi * y / rs, vphi * x / rs, p


def double_rarefaction(x, y, speed=2.0, rho=1.0, p=0.4, split=0.5, band=0.02):
    """(rho, vx, vy, p): uniform gas with vx = -speed for x mod 1 < split and
    +speed above (two gases receding from x = split, colliding at x = 0 mod 1),
    vx = 0 within ``band`` of the collision line; the receding gases open a
    near-vacuum (a strong test of positivity)."""
    xm = np.mod(x, 1.0)
    vx = np.where(xm < split, -speed, speed)
    vx = np.where((xm < band) | (xm > 1.0 - band), 0.0, vx)
    one = np.ones_like(xm)
    return rho * one, vx, 0.0 * one, p * one


def ring_radius(seed):
    """r_ring ~ U[1.4, 1.9] from the seed (index 2**62 + 1 is reserved for it)."""
    return 1.4 + 0.5 * float(uniform01(seed, (np.uint64(1) << np.uint64(62)) + np.uint64(1)))


def ring_jump(seed):
    """A density and pressure jump for the ring workload: factor f ~ U[1.5, 3]
    inside r < r_j, r_j ~ U[1.2, 2.0] (indices 2**62 + 2 and + 3 of the seed)."""
    base = np.uint64(1) << np.uint64(62)
    r_j = 1.2 + 0.8 * float(uniform01(seed, base + np.uint64(2)))
    f = 1.5 + 1.5 * float(uniform01(seed, base + np.uint64(3)))
    return r_j, f


def apply_jump(prim, x, y, r_j, f):
    """prim [var][E][n^2] of an adiabatic state (rho, vx, vy, p) with density
    and pressure multiplied by f at the nodes inside r < r_j (velocity kept)."""
    inside = np.sqrt(np.asarray(x) ** 2 + np.asarray(y) ** 2) < r_j
    out = prim.copy()
    out[0] = np.where(inside, f * prim[0], prim[0])
    out[3] = np.where(inside, f * prim[3], prim[3])
    return out


def pack_prim(fields, n_elem, n_nodes):
    """Stack primitive fields given per node as [E, n^2] into [var][E][n^2]."""
    out = np.empty((len(fields), n_elem, n_nodes), dtype=np.float64)
    for k, f in enumerate(fields):
        out[k] = np.asarray(f, dtype=np.float64).reshape(n_elem, n_nodes)
    return out
