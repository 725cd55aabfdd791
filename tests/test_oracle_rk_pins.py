"""Pins of the oracle's Appendix A time integrators (SSP(2,2), SSP(5,4),
Cash-Karp) against the printed tables and the textbook order conditions.

The order conditions are the rooted-tree conditions of Butcher's theory
(Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.2), listed here up to order
five; they are checked on the oracle's tables, not re-derived from them.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rk_tables_printed.txt")
KIND = {"ssp33": 0, "ssp22": 1, "ssp54": 2, "cashkarp": 3}
ORDER = {"ssp33": 3, "ssp22": 2, "ssp54": 4, "cashkarp": 5}


def _num(tok):
    return float(Fraction(tok)) if "/" in tok else float(tok)


def printed_tables():
    out, name = {}, None
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "table":
                name, s = tok[1], int(tok[2])
                out[name] = {"A": np.zeros((s, s)), "c": np.zeros(s), "b": None, "row": 0}
            elif tok[0] == "b":
                out[name]["b"] = np.array([_num(t) for t in tok[1:]])
            else:
                t = out[name]
                i = t["row"]
                t["c"][i] = _num(tok[0])
                for j, v in enumerate(tok[1:]):
                    t["A"][i, j] = _num(v)
                t["row"] += 1
    return out


def order_conditions(A, b, c):
    """(order, residual) of each tree condition up to order five."""
    e = np.ones_like(c)
    Ac = A @ c
    rows = [
        (1, b @ e - 1),
        (2, b @ c - 1 / 2),
        (3, b @ c ** 2 - 1 / 3), (3, b @ Ac - 1 / 6),
        (4, b @ c ** 3 - 1 / 4), (4, b @ (c * Ac) - 1 / 8), (4, b @ (A @ c ** 2) - 1 / 12),
        (4, b @ (A @ Ac) - 1 / 24),
        (5, b @ c ** 4 - 1 / 5), (5, b @ (c ** 2 * Ac) - 1 / 10), (5, b @ (c * (A @ c ** 2)) - 1 / 15),
        (5, b @ (c * (A @ Ac)) - 1 / 30), (5, b @ (Ac * Ac) - 1 / 20), (5, b @ (A @ c ** 3) - 1 / 20),
        (5, b @ (A @ (c * Ac)) - 1 / 40), (5, b @ (A @ (A @ c ** 2)) - 1 / 60),
        (5, b @ (A @ (A @ Ac)) - 1 / 120),
    ]
    return rows


def test_printed_tables_match_the_oracle_where_taken_as_printed():
    pr = printed_tables()
    for name in ("ssp54", "cashkarp"):
        A, b, c = O.rk_tableau(KIND[name])
        assert np.array_equal(A, pr[name]["A"]), name
        assert np.array_equal(b, pr[name]["b"]), name
        assert np.array_equal(c, pr[name]["c"]), name


def test_printed_ssp22_is_first_order_and_the_reading_is_heun():
    pr = printed_tables()["ssp22"]
    assert abs(pr["b"] @ pr["c"] - 0.5) > 0.2  # the printed table fails order two
    A, b, c = O.rk_tableau(KIND["ssp22"])
    assert np.array_equal(b, pr["b"])
    assert A[1, 0] == 1.0 and c[1] == 1.0  # a_21 = c_2 = 1 (Heun)
    # Heun is the convex combination of two forward-Euler steps (SSP)
    z = -0.7
    y = O.rk_butcher(A, b, c, lambda t, y: z * y, np.array([1.0]), 0.0, 1.0)
    assert abs(y[0] - 0.5 * (1 + (1 + z) * (1 + z))) < 1e-16


@pytest.mark.parametrize("name", ["ssp22", "ssp33", "ssp54", "cashkarp"])
def test_order_conditions(name):
    A, b, c = O.rk_tableau(KIND[name])
    p = ORDER[name]
    # printed 14-digit decimals of the five-stage table: consistent to ~1e-10
    tol = 2e-10 if name == "ssp54" else 1e-15
    assert np.max(np.abs(A.sum(axis=1) - c)) <= (2e-14 if name == "ssp54" else 3e-16)
    assert np.allclose(np.tril(A, -1), A, atol=0)  # explicit
    for order, res in order_conditions(A, b, c):
        if order <= p:
            assert abs(res) <= tol, (name, order, res)
    # and not of order p + 1 (at least one condition of the next order fails)
    nxt = [abs(r) for o, r in order_conditions(A, b, c) if o == p + 1]
    if nxt:
        assert max(nxt) > 1e-4, name


@pytest.mark.parametrize("name", ["ssp22", "ssp33", "ssp54", "cashkarp"])
def test_observed_order_on_a_nonlinear_nonautonomous_ode(name):
    # y' = -2 t y^2, y(0) = 1: y = 1 / (1 + t^2); integrate to t = 2
    A, b, c = O.rk_tableau(KIND[name])
    f = lambda t, y: -2.0 * t * y * y  # noqa: E731

    def err(nsteps):
        y, t, h = np.array([1.0]), 0.0, 2.0 / nsteps
        for _ in range(nsteps):
            y = O.rk_butcher(A, b, c, f, y, t, h)
            t += h
        return abs(y[0] - 1.0 / (1.0 + t * t))

    e1, e2 = err(20), err(40)
    rate = np.log2(e1 / e2)
    assert ORDER[name] - 0.35 < rate < ORDER[name] + 0.6, (name, e1, e2, rate)


@pytest.mark.parametrize("rk", [1, 2, 3])
def test_dg_step_uses_the_chosen_table(rk):
    # one oracle DG step with the table of `rk` against the Butcher stages
    # written with the oracle's L(u): the planet moves between stages, so the
    # stage times are pinned too
    c = O.cfg(n=3, nvar=3, nx=6, ny=6, x0=-2.5, x1=2.5, y0=-2.5, y1=2.5, closure=1, h=0.05, bc=0,
              star=1, q=1e-3, eps=0.3, damping=0, rk=rk)
    from paper_1805_01443_amd import synth as S
    x, y = O.nodes(c)
    sig, vx, vy = S.disc(x, y, h=0.05)
    u = O.project(c, S.pack_prim((sig, vx, vy), 36, 9))
    A, b, cc = O.rk_tableau(rk)
    t0, dt = 0.2, 0.01
    ks = []
    for i in range(len(b)):
        yi = u + dt * sum(A[i, j] * ks[j] for j in range(i))
        ks.append(O.rhs(c, t0 + cc[i] * dt, yi))
    want = u + dt * sum(b[i] * ks[i] for i in range(len(b)))
    got, d = O.step(c, u, t0, dt)
    assert d == dt
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


def test_unknown_table_is_rejected():
    with pytest.raises(ValueError):
        O.rk_tableau(9)
