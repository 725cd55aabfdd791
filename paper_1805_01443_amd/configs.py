"""The workloads of this implementation, as configurations plus initial data.

* ``wave``      order 3 (P2), isothermal c_s = 1, 64 x 64 periodic unit square,
                rho = 1 + 0.2 sin(2 pi (x + y)), v = (1, 1), CFL 0.2, 100 steps.
* ``disc``      order 5 (P4), locally isothermal h = 0.05, 512 x 512 on
                [-2.5, 2.5]^2, Sigma = Sigma0 r^(-1/2) in rotational equilibrium,
                damping for r < 0.4 and r > 2.3, planet q = 1e-5 at r = 1 with
                softening 0.6 H = 0.03; 200 steps, torque every step.
* ``disc_sweep``  the disc at 1024 x 1024, orders 2..5, q = 3e-5, Sigma0 and a
                1e-4 density noise drawn from a seed.
* ``disc_mixed``  the sweep disc at order 5 in the mixed-precision deviation form.
* ``disc_ring``   the adiabatic disc at order 4 with an over-pressure ring, for
                the troubled-cell indicator.
* ``rarefaction`` adiabatic gases receding at Mach 2.7 on a periodic strip,
                with the positivity-preserving limiter.
* ``vortex``      the isentropic vortex of Sec. 4.1 (beta = 5, gamma = 1.4) on the
                periodic box [0, 10]^2.
* ``gresho``      the Gresho vortex of Sec. 4.2 on [0, 1]^2 with gradient-free
                box edges, gamma = 1.4.
* ``paper_disc``  the adiabatic disc of Sec. 5.1: box [-2.25, 2.25]^2, Sigma0 = 1,
                p0 = 2.5e-3, r_in = 0.4, r_ex = 1.75, gamma = 1.4, planet q = 6e-5
                with softening 0.03, damping radii r_in 1.15^(3/2) and
                r_ex 1.15^(-3/2).
"""
from __future__ import annotations

import numpy as np

from . import synth
from .dg import (BC_FIXED_INITIAL, BC_GRADIENT_FREE, BC_PERIODIC, CLOSURE_ADIABATIC, CLOSURE_ISOTHERMAL,
                 CLOSURE_LOCALLY_ISOTHERMAL, PRECISION_MIXED, Config, dg_get_nodes)


def wave(nx=64, order=3):
    return Config(order=order, nvar=3, nx=nx, ny=nx, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                  closure=CLOSURE_ISOTHERMAL, cs=1.0, bc=BC_PERIODIC, cfl=0.2)


def disc(nx=512, order=5, q=1e-5, h=0.05):
    return Config(order=order, nvar=3, nx=nx, ny=nx, x0=-2.5, x1=2.5, y0=-2.5, y1=2.5,
                  closure=CLOSURE_LOCALLY_ISOTHERMAL, h=h, bc=BC_FIXED_INITIAL, star=1, gm=1.0,
                  r_core=0.4, q=q, eps=0.6 * h, rp=1.0, phi0=0.0, damping=1, rd_in=0.4, rd_out=2.3,
                  cfl=0.2)


def disc_sweep(nx=1024, order=5):
    return disc(nx=nx, order=order, q=3e-5)


def disc_mixed(nx=1024, order=5, seed=0, q=3e-5):
    """The sweep disc in the mixed-precision deviation form about the
    equilibrium with the seed's Sigma0."""
    return disc(nx=nx, order=order, q=q).replace(precision=PRECISION_MIXED, sigma0=sigma0_of(seed))


def disc_ring(nx=1024, order=4):
    c = disc(nx=nx, order=order, q=3e-5)
    return c.replace(nvar=4, closure=CLOSURE_ADIABATIC, gamma=1.4)


def rarefaction(nx=32, ny=2, order=3):
    return Config(order=order, nvar=4, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=ny / nx,
                  closure=CLOSURE_ADIABATIC, gamma=1.4, bc=BC_PERIODIC, cfl=1.0, positivity=1)


def vortex(nx=40, order=3):
    return Config(order=order, nvar=4, nx=nx, ny=nx, x0=0.0, x1=10.0, y0=0.0, y1=10.0,
                  closure=CLOSURE_ADIABATIC, gamma=1.4, bc=BC_PERIODIC, cfl=0.2)


def gresho(nx=40, order=3):
    return Config(order=order, nvar=4, nx=nx, ny=nx, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                  closure=CLOSURE_ADIABATIC, gamma=1.4, bc=BC_GRADIENT_FREE, cfl=0.2)


def paper_disc(nx=320, order=5, q=6e-5, positivity=1):
    """With the paper's positivity-preserving limiter (Sec. 2.4): the disc's
    outer taper leaves densities down to 1e-13 in the box corners."""
    f = 1.15 ** 1.5
    return Config(order=order, nvar=4, nx=nx, ny=nx, x0=-2.25, x1=2.25, y0=-2.25, y1=2.25,
                  closure=CLOSURE_ADIABATIC, gamma=1.4, h=0.05, bc=BC_FIXED_INITIAL, star=1, gm=1.0,
                  r_core=0.4, q=q, eps=0.03, rp=1.0, phi0=0.0, damping=1, rd_in=0.4 * f, rd_out=1.75 / f,
                  cfl=0.2, positivity=positivity)


def prim_for(cfg: Config, kind: str, seed=None, x=None, y=None):
    """Primitive node values [var][E][n^2] of a workload.  Node coordinates
    default to the library's (dg_get_nodes); tests pass the oracle's."""
    if x is None:
        x, y = dg_get_nodes(cfg)
    E, nn = cfg.n_elem, cfg.order ** 2
    if kind == "wave":
        fields = synth.periodic_wave(x, y)
    elif kind == "disc":
        s0 = 1.0 if seed is None else synth.disc_sigma0(seed)
        fields = synth.disc(x, y, gm=cfg.gm, h=cfg.h, r_core=cfg.r_core, sigma0=s0,
                            noise_seed=seed, noise_amp=1e-4)
    elif kind == "disc_eq":
        s0 = 1.0 if seed is None else synth.disc_sigma0(seed)
        fields = synth.disc(x, y, gm=cfg.gm, h=cfg.h, r_core=cfg.r_core, sigma0=s0)
    elif kind == "disc_ring":
        s0 = 1.0 if seed is None else synth.disc_sigma0(seed)
        rr = 1.6 if seed is None else synth.ring_radius(seed)
        fields = synth.disc_ring(x, y, gm=cfg.gm, h=cfg.h, r_core=cfg.r_core, sigma0=s0, r_ring=rr)
    elif kind == "rarefaction":
        fields = synth.double_rarefaction(x, y)
    elif kind == "vortex":
        fields = synth.isentropic_vortex(x, y)
    elif kind == "gresho":
        fields = synth.gresho(x, y)
    elif kind == "paper_disc":
        fields = synth.paper_disc(x, y, gm=cfg.gm, r_in=cfg.r_core)
    else:
        raise ValueError(kind)
    return synth.pack_prim(fields, E, nn)


def dofs(cfg: Config) -> int:
    """Degrees of freedom n_x n_y m^2 (Sec. 3.1)."""
    return cfg.nx * cfg.ny * cfg.order ** 2


def sigma0_of(seed):
    return 1.0 if seed is None else synth.disc_sigma0(seed)


__all__ = ["wave", "disc", "disc_sweep", "disc_ring", "rarefaction", "vortex", "gresho", "paper_disc", "prim_for", "dofs", "np"]
