"""Pins of the oracle's troubled-cell parts (indicator, minmod limiter, MLP,
loss, Adam) against closed forms, invariants and independent library routines
(PyTorch CPU autograd, BCE-with-logits, Adam and its bfloat16 cast)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1805_01443_amd import synth as S


def _cfg(n=4, nx=8, ny=6, nvar=4, **kw):
    d = dict(n=n, nx=nx, ny=ny, nvar=nvar, closure=2 if nvar == 4 else 0)
    d.update(kw)
    return O.cfg(**d)


# ---------------------------------------------------------------- indicator
def test_indicator_closed_forms():
    c = _cfg(n=4, nx=3, ny=2)
    E, nn = 6, 16
    u = np.zeros((4, nn, E))
    u[0, 0, :] = 2.0
    u[0, 1 * 4 + 1, 0] = 0.3      # degree (1,1): below the top degree
    u[0, 3 * 4 + 0, 1] = 0.5      # (3,0): top degree in x
    u[0, 2 * 4 + 3, 2] = 0.1      # (2,3): top degree in y
    u[0, 3 * 4 + 3, 3] = 1.0      # (3,3)
    s = O.indicator(c, u)
    assert s[0] == -300.0 and s[4] == -300.0
    assert abs(s[1] - math.log10(0.25 / (4.0 + 0.25))) < 1e-14
    assert abs(s[2] - math.log10(0.01 / 4.01)) < 1e-14
    assert abs(s[3] - math.log10(1.0 / 5.0)) < 1e-14
    s2 = O.indicator(c, 3.0 * u)
    assert np.allclose(s2, s, rtol=0, atol=1e-14)  # scale invariant


def test_indicator_step_vs_legendre_coefficients():
    """A density jump inside one element: its top-degree energy share equals
    the closed-form Legendre coefficients of the step (numpy quadrature)."""
    n = 4
    c = _cfg(n=n, nx=1, ny=1, x0=-1, x1=1, y0=-1, y1=1)
    # exact modal coefficients of H(xi) (times 1 in eta) for the normalised basis:
    # u_a = (1/2) int_0^1 phi_a(xi) dxi
    xs, ws = np.polynomial.legendre.leggauss(40)
    xg = 0.5 * (xs + 1.0)
    wg = 0.5 * ws
    coef = []
    for a in range(n):
        ca = np.zeros(a + 1)
        ca[a] = math.sqrt(2 * a + 1)
        coef.append(0.5 * np.sum(wg * np.polynomial.legendre.legval(xg, ca)))
    u = np.zeros((4, n * n, 1))
    for a in range(n):
        u[0, a * n, 0] = 1.0 * (a == 0) + coef[a]
    s = O.indicator(c, u)
    tot = (1.0 + coef[0]) ** 2 + sum(cc * cc for cc in coef[1:])
    assert abs(s[0] - math.log10(coef[n - 1] ** 2 / tot)) < 1e-12


# ---------------------------------------------------------------- minmod
def _linear_state(c, alpha=0.7, beta=-0.3):
    X, Y = O.nodes(c)
    rho = 2.0 + alpha * X + beta * Y
    f = [rho, 0.1 + 0 * X, -0.2 + 0 * X, 3.0 + 0 * X]
    return O.project(c, S.pack_prim(f[:c.nvar], X.shape[0], c.n * c.n)), X, Y


def test_minmod_keeps_linear_data_and_means():
    c = _cfg(n=3, nx=8, ny=6, nvar=4, bc=0)
    u, _, _ = _linear_state(c)
    # interior elements (periodic wrap breaks linearity at the box edge)
    E = 48
    inner = np.array([e for e in range(E) if 0 < e % 8 < 7 and 0 < e // 8 < 5])
    flags = np.zeros(E, bool)
    flags[inner] = True
    ul, ch = O.minmod(c, u, u, flags)
    assert not ch[inner].any()
    assert np.array_equal(ul, u)


def test_minmod_step_function_tvd_slopes():
    n = 3
    c = _cfg(n=n, nx=10, ny=2, nvar=4, bc=1, x0=0, x1=1, y0=0, y1=0.2)
    X, Y = O.nodes(c)
    rho = np.where(X < 0.5, 1.0, 0.2) + 0.3 * X   # jump plus a linear ramp
    f = [rho, 0 * X, 0 * X, 1.0 + 0 * X]
    u = O.project(c, S.pack_prim(f, X.shape[0], n * n))
    # an element that straddles nothing: move the jump inside element 4 by shifting
    X2 = X.copy()
    rho2 = np.where(X2 < 0.45, 1.0, 0.2) + 0.3 * X2
    u = O.project(c, S.pack_prim([rho2, 0 * X, 0 * X, 1.0 + 0 * X], X.shape[0], n * n))
    flags = np.ones(c.nx * c.ny, bool)
    ul, ch = O.minmod(c, u, u, flags)
    E = c.nx * c.ny
    m = u[0, 0]
    assert np.array_equal(ul[:, 0], u[:, 0])  # means untouched bitwise
    e = 4  # the element holding the jump (x in [0.4, 0.5])
    assert ch[e]
    sx = math.sqrt(3.0) * ul[0, 1 * n + 0, e]
    dr = m[e + 1] - m[e]
    dl = m[e] - m[e - 1]
    a = math.sqrt(3.0) * u[0, 1 * n + 0, e]
    expect = 0.0 if not (a * dr > 0 and a * dl > 0) else math.copysign(min(abs(a), abs(dr), abs(dl)), a)
    assert abs(sx - expect) < 1e-15
    # higher modes dropped in limited elements
    assert np.all(ul[:, 2, ch] == 0.0) and np.all(ul[:, n + 1, ch] == 0.0)
    # unflagged elements untouched
    fl2 = np.zeros(E, bool)
    ul2, ch2 = O.minmod(c, u, u, fl2)
    assert np.array_equal(ul2, u) and not ch2.any()


def test_limited_step_without_flags_equals_unlimited_step():
    c = _cfg(n=3, nx=8, ny=8, nvar=3, closure=0)
    X, Y = O.nodes(c)
    u = O.project(c, S.pack_prim(S.periodic_wave(X, Y), 64, 9))
    a, da = O.step_limited(c, u, 0.1, 1e-3, u, s0=1e9)
    b, db = O.step(c, u, 0.1, 1e-3)
    assert da == db and np.max(np.abs(a - b)) < 1e-14


def test_limited_step_conserves_mass():
    c = _cfg(n=4, nx=12, ny=10, nvar=4, bc=0)
    X, Y = O.nodes(c)
    rho = np.where((X - 0.5) ** 2 + (Y - 0.5) ** 2 < 0.05, 2.0, 1.0)
    f = [rho, 0.3 + 0 * X, 0.1 + 0 * X, 2.0 + 0 * X]
    u = O.project(c, S.pack_prim(f, X.shape[0], 16))
    s = O.indicator(c, u)
    s0 = float(np.median(s))
    un, _ = O.step_limited(c, u, 0.0, 2e-4, u, s0=s0)
    assert abs(un[0, 0].sum() - u[0, 0].sum()) < 1e-13 * u[0, 0].sum()


def test_limited_step_limits_after_every_stage():
    """Sec. 3.1 (iii)(d): the limiter acts inside every Runge-Kutta sub-step.
    The oracle's limited step equals the SSP(3,3) Shu-Osher stages with the
    indicator + minmod applied to each stage state (composed here from the
    separately pinned right-hand side, indicator and minmod), and differs from
    limiting only the end state of an unlimited step."""
    n = 3
    c = _cfg(n=n, nx=14, ny=12, nvar=4, bc=0, x0=0, x1=1, y0=0, y1=1)
    X, Y = O.nodes(c)
    # a steep (unresolved) density front, uniform pressure 1
    rho = 2.0 - np.tanh((np.sqrt((X - 0.45) ** 2 + (Y - 0.55) ** 2) - 0.245) / 0.03)
    f = [rho, 0.4 * rho, -0.2 * rho, 1.0 / 0.4 + 0.5 * rho * (0.16 + 0.04)]
    u = O.project(c, S.pack_prim(f, X.shape[0], n * n))
    s0 = float(np.quantile(O.indicator(c, u), 0.7))
    dt, t = 4e-3, 0.2

    def lim(w):
        return O.minmod(c, w, u, O.indicator(c, w) > s0)[0]

    u1 = lim(u + dt * O.rhs(c, t, u))
    u2 = lim(0.75 * u + 0.25 * (u1 + dt * O.rhs(c, t + dt, u1)))
    u3 = lim(u / 3.0 + 2.0 / 3.0 * (u2 + dt * O.rhs(c, t + 0.5 * dt, u2)))
    got, d = O.step_limited(c, u, t, dt, u, s0)
    assert d == dt
    assert np.max(np.abs(got - u3)) <= 1e-15 * np.max(np.abs(u3))
    # the stage limiting changes the result: limiting only at the end differs
    end_only = lim(O.step(c, u, t, dt)[0])
    assert np.max(np.abs(end_only - got)) > 1e-6 * np.max(np.abs(got))
    # and the intermediate stage states were flagged and changed
    assert (O.indicator(c, u + dt * O.rhs(c, t, u)) > s0).sum() > 0
    assert O.minmod(c, u + dt * O.rhs(c, t, u), u, O.indicator(c, u + dt * O.rhs(c, t, u)) > s0)[1].any()


def test_mlp_features_hand_built_state():
    """Feature definition u_vm / (|u_v00| + s_v), index v * n^2 + m with the
    flat mode m = a * n + b (a: degree in x): two hand-built elements."""
    n = 4
    c = _cfg(n=n, nx=2, ny=1, nvar=4)
    u = np.zeros((4, n * n, 2))
    # element 0: negative density mean (the absolute value enters), distinct
    # x- and y-slopes so a transposed mode index is seen
    u[0, 0, 0] = -2.0
    u[0, 1 * n + 0, 0] = 0.5     # mode (1, 0)
    u[0, 0 * n + 1, 0] = -0.25   # mode (0, 1)
    u[3, 0, 0] = 4.0
    u[3, 3 * n + 2, 0] = 1.5     # mode (3, 2) of the energy
    # element 1: zero mean, the scale alone normalises
    u[1, 2 * n + 1, 1] = 0.3     # mode (2, 1) of x-momentum
    scale = np.array([0.5, 0.25, 1.0, 2.0])
    f = O.mlp_features(c, u, scale)
    assert f.shape == (2, 64)
    assert f[0, 0] == -2.0 / 2.5
    assert f[0, 0 * 16 + 4] == 0.5 / 2.5      # v = 0, m = 1 * 4 + 0
    assert f[0, 0 * 16 + 1] == -0.25 / 2.5    # v = 0, m = 0 * 4 + 1
    assert f[0, 3 * 16 + 0] == 4.0 / 6.0
    assert f[0, 3 * 16 + 14] == 1.5 / 6.0     # v = 3, m = 3 * 4 + 2
    assert f[1, 1 * 16 + 9] == 0.3 / 0.25     # v = 1, m = 2 * 4 + 1
    nz = {(0, 0), (0, 4), (0, 1), (0, 48), (0, 62), (1, 25)}
    for e in range(2):
        for k in range(64):
            if (e, k) not in nz:
                assert f[e, k] == 0.0, (e, k)


# ---------------------------------------------------------------- MLP
def _params(seed=0):
    rng = np.random.default_rng(seed)
    p = np.zeros(O.MLP_NPARAM)
    p[:2048] = rng.normal(0, 1 / 8, 2048)
    p[2048:2080] = rng.normal(0, 0.1, 32)
    p[2080:3104] = rng.normal(0, 1 / math.sqrt(32), 1024)
    p[3104:3136] = rng.normal(0, 0.1, 32)
    p[3136:3168] = rng.normal(0, 1 / math.sqrt(32), 32)
    p[3168] = 0.05
    return p


def _torch_mlp(p, x, y=None, pos_weight=1.0):
    import torch
    P = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    W1 = P[:2048].view(32, 64)
    b1 = P[2048:2080]
    W2 = P[2080:3104].view(32, 32)
    b2 = P[3104:3136]
    w3 = P[3136:3168]
    b3 = P[3168]
    X = torch.tensor(x, dtype=torch.float64)
    h1 = torch.relu(X @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    z = h2 @ w3 + b3
    if y is None:
        return z.detach().numpy()
    loss = torch.nn.functional.binary_cross_entropy_with_logits(
        z, torch.tensor(y, dtype=torch.float64), pos_weight=torch.tensor(pos_weight, dtype=torch.float64))
    loss.backward()
    return loss.item(), P.grad.numpy()


def test_mlp_forward_and_gradient_match_torch_fp64():
    rng = np.random.default_rng(1)
    p = _params(1)
    x = rng.normal(0, 1, (257, 64))
    y = (rng.random(257) < 0.2).astype(float)
    z, _, _ = O.mlp_forward(p, x, bf16=False)
    assert np.max(np.abs(z - _torch_mlp(p, x))) < 1e-13
    loss, g = O.mlp_loss_grad(p, x, y, pos_weight=3.5, bf16=False)
    lt, gt = _torch_mlp(p, x, y, 3.5)
    assert abs(loss - lt) < 1e-13
    assert np.max(np.abs(g - gt)) < 1e-13 * max(1.0, np.max(np.abs(gt)))


def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(2)
    p = _params(2)
    x = rng.normal(0, 1, (16, 64))
    y = (rng.random(16) < 0.5).astype(float)
    _, g = O.mlp_loss_grad(p, x, y, pos_weight=2.0, bf16=False)
    for k in list(range(0, 3169, 97)) + [3168, 3136, 2080, 2048]:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (O.mlp_loss_grad(pp, x, y, 2.0, False)[0] - O.mlp_loss_grad(pm, x, y, 2.0, False)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.normal(0, 10, 2000), [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.4e38, 1e-40]])
    ref = torch.tensor(xs, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([O.bf16(v) for v in xs])
    assert np.array_equal(got, ref)


def test_bf16_forward_close_to_fp64_forward():
    rng = np.random.default_rng(4)
    p = _params(4)
    x = rng.normal(0, 1, (128, 64))
    z16, _, _ = O.mlp_forward(p, x, bf16=True)
    z64, _, _ = O.mlp_forward(p, x, bf16=False)
    assert np.max(np.abs(z16 - z64)) < 0.05 * np.max(np.abs(z64))  # bf16 has 8 significant bits


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(5)
    p = rng.normal(0, 1, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    P = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([P], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(0, 1, 50)
        p, m, v = O.adam(p, g, m, v, t)
        opt.zero_grad()
        P.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    assert np.max(np.abs(p - P.detach().numpy())) < 1e-14
