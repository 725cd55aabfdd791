/*
 * Plain FP64 CPU oracle for the modal DG scheme of Velasco Romero et al. (2018).
 *
 * TEST INFRASTRUCTURE ONLY -- see dg_oracle.h.  Every routine below follows
 * the paper's statement of the method directly: nodal values are evaluated by
 * the full double sum over modes, every integral of eq. (3) is its quadrature
 * sum written out, each element computes the numerical flux on its own four
 * edges with its own outward normal, and time stepping uses the Butcher form
 * of Algorithm 1.  No sum factorisation, no fusion, no reordering.
 *
 * Readings of points the paper leaves open (numerical flux type, stellar
 * potential inside r_core, exterior state at the box edge, damping radii,
 * torque cell masses) are the ones listed with the design notes; each is
 * named where it is used.
 */
#include "dg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 8
#define OR_MAXV 4

/* ------------------------------------------------------------------ */
/* Legendre polynomials and Gauss-Legendre quadrature (Sec. 2.2)       */
/* ------------------------------------------------------------------ */

/* P_a(x) by Bonnet's recursion (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1} */
static double legendre_p(int a, double x)
{
    double p0 = 1.0, p1 = x;
    if (a == 0) return 1.0;
    for (int k = 1; k < a; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

/* P_a'(x) from P'_{k+1} = P'_{k-1} + (2k+1) P_k */
static double legendre_dp(int a, double x)
{
    if (a == 0) return 0.0;
    double dm1 = 0.0, d0 = 1.0; /* P'_0, P'_1 */
    for (int k = 1; k < a; ++k) {
        double d1 = dm1 + (2.0 * k + 1.0) * legendre_p(k, x);
        dm1 = d0;
        d0 = d1;
    }
    return d0;
}

/* basis normalised so that (1/|K|) int_K phi_ab phi_cd = delta (mean = mode 00) */
double or_phi(int a, double x) { return sqrt(2.0 * a + 1.0) * legendre_p(a, x); }
double or_dphi(int a, double x) { return sqrt(2.0 * a + 1.0) * legendre_dp(a, x); }

/* Newton iteration on P_n from the Chebyshev-like first guess; weights
 * w = 2 / ((1 - x^2) P_n'(x)^2).  Nodes come out ascending and symmetric. */
int or_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > OR_MAXN) return -1;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(pi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double dz = legendre_p(n, z) / legendre_dp(n, z);
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        if (2 * i + 1 == n) z = 0.0;
        double dp = legendre_dp(n, z);
        double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        x[n - 1 - i] = z;
        x[i] = (2 * i + 1 == n) ? 0.0 : -z;
        w[n - 1 - i] = wi;
        w[i] = wi;
    }
    return 0;
}

int or_gauss_lobatto(int L, double *x, double *w)
{
    if (L < 2 || L > OR_MAXN + 1) return -1;
    const double pi = 3.14159265358979323846;
    int k = L - 1; /* interior nodes: roots of P_k' */
    for (int i = 0; i < L; ++i) {
        double z;
        if (i == 0)
            z = -1.0;
        else if (i == k)
            z = 1.0;
        else {
            z = -cos(pi * i / k); /* Chebyshev-Gauss-Lobatto start */
            for (int it = 0; it < 100; ++it) {
                /* Newton on P_k'; P_k'' from Legendre's equation
                 * (1 - z^2) P'' = 2 z P' - k (k+1) P */
                double d1 = legendre_dp(k, z);
                double d2 = (2.0 * z * d1 - k * (k + 1.0) * legendre_p(k, z)) / (1.0 - z * z);
                double dz = d1 / d2;
                z -= dz;
                if (fabs(dz) < 1e-17) break;
            }
            if (2 * i == k) z = 0.0;
        }
        double pk = legendre_p(k, z);
        x[i] = z;
        w[i] = 2.0 / (k * (k + 1.0) * pk * pk);
    }
    return 0;
}

int or_pp_lobatto_points(int np)
{
    int L = 2;
    while (2 * L - 3 < np) ++L;
    return L;
}

/* ------------------------------------------------------------------ */
/* per-configuration tables                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int n, nn;
    double xi[OR_MAXN], wh[OR_MAXN];          /* nodes and weights / 2 */
    double phi[OR_MAXN][OR_MAXN];             /* phi[a][q] = phi_a(xi_q) */
    double dphi[OR_MAXN][OR_MAXN];            /* dphi[a][q] = phi_a'(xi_q) */
    double dx, dy;
} tables;

static void make_tables(const or_cfg *c, tables *T)
{
    double w[OR_MAXN];
    T->n = c->n;
    T->nn = c->n * c->n;
    or_gauss_legendre(c->n, T->xi, w);
    for (int q = 0; q < c->n; ++q) T->wh[q] = 0.5 * w[q];
    for (int a = 0; a < c->n; ++a)
        for (int q = 0; q < c->n; ++q) {
            T->phi[a][q] = or_phi(a, T->xi[q]);
            T->dphi[a][q] = or_dphi(a, T->xi[q]);
        }
    T->dx = (c->x1 - c->x0) / c->nx;
    T->dy = (c->y1 - c->y0) / c->ny;
}

static double elem_xc(const or_cfg *c, const tables *T, int i) { return c->x0 + (i + 0.5) * T->dx; }
static double elem_yc(const or_cfg *c, const tables *T, int j) { return c->y0 + (j + 0.5) * T->dy; }

void or_nodes(const or_cfg *c, double *x, double *y)
{
    tables T;
    make_tables(c, &T);
    long E = (long)c->nx * c->ny;
    for (long e = 0; e < E; ++e) {
        int i = (int)(e % c->nx), j = (int)(e / c->nx);
        for (int q = 0; q < c->n; ++q)
            for (int r = 0; r < c->n; ++r) {
                x[e * T.nn + q * c->n + r] = elem_xc(c, &T, i) + 0.5 * T.dx * T.xi[q];
                y[e * T.nn + q * c->n + r] = elem_yc(c, &T, j) + 0.5 * T.dy * T.xi[r];
            }
    }
}

/* u_h at reference point (xi, eta) of element e: sum_ab u_ab phi_a(xi) phi_b(eta) */
static void eval_point(const or_cfg *c, const double *u, long e, double xi, double eta, double *U)
{
    long E = (long)c->nx * c->ny;
    int n = c->n;
    for (int v = 0; v < c->nvar; ++v) {
        double s = 0.0;
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                s += u[((long)v * n * n + a * n + b) * E + e] * or_phi(a, xi) * or_phi(b, eta);
        U[v] = s;
    }
}

void or_eval_nodes(const or_cfg *c, const double *u, double *out)
{
    tables T;
    make_tables(c, &T);
    long E = (long)c->nx * c->ny;
    int n = c->n;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int v = 0; v < c->nvar; ++v) {
                    double s = 0.0;
                    for (int a = 0; a < n; ++a)
                        for (int b = 0; b < n; ++b)
                            s += u[((long)v * T.nn + a * n + b) * E + e] * T.phi[a][q] * T.phi[b][r];
                    out[((long)v * E + e) * T.nn + q * n + r] = s;
                }
    }
}

/* ------------------------------------------------------------------ */
/* physics: closure, flux, gravity (Sec. 2.1 eq. (1); Sec. 5.1)         */
/* ------------------------------------------------------------------ */

void or_planet_pos(const or_cfg *c, double t, double *xp, double *yp)
{
    /* fixed circular orbit; G = M_* = 1 units give Omega_p = sqrt(GM / r_p^3) */
    double om = sqrt(c->gm / (c->rp * c->rp * c->rp));
    *xp = c->rp * cos(om * t + c->phi0);
    *yp = c->rp * sin(om * t + c->phi0);
}

/* pressure and sound speed of the conservative state U at (x, y) */
static void closure(const or_cfg *c, const double *U, double x, double y, double *p, double *cs)
{
    if (c->closure == 0) {
        *p = c->cs * c->cs * U[0];
        *cs = c->cs;
    } else if (c->closure == 1) {
        double r = sqrt(x * x + y * y);
        double cs2 = c->h * c->h * c->gm / (r > c->r_core ? r : c->r_core);
        *p = cs2 * U[0];
        *cs = sqrt(cs2);
    } else {
        double ke = 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0];
        *p = (c->gamma - 1.0) * (U[3] - ke);
        *cs = sqrt(c->gamma * *p / U[0]);
    }
}

/* f(U) . (nx, ny) */
static void flux_n(const or_cfg *c, const double *U, double p, double nx, double ny, double *F)
{
    double vn = (U[1] * nx + U[2] * ny) / U[0];
    F[0] = U[0] * vn;
    F[1] = U[1] * vn + p * nx;
    F[2] = U[2] * vn + p * ny;
    if (c->nvar == 4) F[3] = (U[3] + p) * vn;
}

/* grad Phi: stellar potential -GM/r outside r_core and the harmonic core
 * GM (r^2 - 3 r_core^2) / (2 r_core^3) inside (solid rotation there), plus the
 * softened planet -q / sqrt(d^2 + eps^2); no indirect term. */
static void grad_phi(const or_cfg *c, double x, double y, double t, double *gx, double *gy)
{
    *gx = 0.0;
    *gy = 0.0;
    if (c->star) {
        double r = sqrt(x * x + y * y);
        double k = r < c->r_core ? c->gm / (c->r_core * c->r_core * c->r_core) : c->gm / (r * r * r);
        *gx += k * x;
        *gy += k * y;
    }
    if (c->q > 0.0) {
        double xp, yp;
        or_planet_pos(c, t, &xp, &yp);
        double dx = x - xp, dy = y - yp;
        double d2 = dx * dx + dy * dy + c->eps * c->eps;
        double k = c->q / (d2 * sqrt(d2));
        *gx += k * dx;
        *gy += k * dy;
    }
}

/* Rusanov (local Lax-Friedrichs) flux with the outward normal of the element:
 * h = (f(u_in).n + f(u_out).n)/2 - alpha (u_out - u_in)/2,
 * alpha = max(|v_in.n| + c_in, |v_out.n| + c_out). */
static void rusanov(const or_cfg *c, const double *Ui, const double *Uo, double nx, double ny,
                    double x, double y, double *h)
{
    double pi, ci, po, co, Fi[OR_MAXV], Fo[OR_MAXV];
    closure(c, Ui, x, y, &pi, &ci);
    closure(c, Uo, x, y, &po, &co);
    flux_n(c, Ui, pi, nx, ny, Fi);
    flux_n(c, Uo, po, nx, ny, Fo);
    double si = fabs((Ui[1] * nx + Ui[2] * ny) / Ui[0]) + ci;
    double so = fabs((Uo[1] * nx + Uo[2] * ny) / Uo[0]) + co;
    double alpha = si > so ? si : so;
    for (int v = 0; v < c->nvar; ++v) h[v] = 0.5 * (Fi[v] + Fo[v]) - 0.5 * alpha * (Uo[v] - Ui[v]);
}

/* HLLC flux for the adiabatic closure (Toro, Spruce & Speares 1994; Toro,
 * Riemann Solvers and Numerical Methods for Fluid Dynamics, Sec. 10.4), left
 * state = the element's own trace, right state = the exterior, n = the
 * element's outward normal; normal velocities q = v.n.  Wave speeds as
 * estimated by Davis (1988):
 *   S_L = min(q_L - c_L, q_R - c_R),  S_R = max(q_L + c_L, q_R + c_R);
 * contact speed from the momentum jump conditions across the two outer waves:
 *   S* = (p_R - p_L + rho_L q_L (S_L - q_L) - rho_R q_R (S_R - q_R))
 *        / (rho_L (S_L - q_L) - rho_R (S_R - q_R));
 * star state of side K (density, momentum with the normal velocity replaced by
 * S*, energy):
 *   U*_K = rho_K (S_K - q_K) / (S_K - S*)
 *          [1, v_K + (S* - q_K) n, E_K / rho_K + (S* - q_K) (S* + p_K / (rho_K (S_K - q_K)))];
 * flux: F_L if S_L >= 0; F_L + S_L (U*_L - U_L) if S_L < 0 <= S*;
 * F_R + S_R (U*_R - U_R) if S* < 0 < S_R; F_R if S_R <= 0. */
static void hllc(const or_cfg *c, const double *UL, const double *UR, double nx, double ny, double x, double y,
                 double *h)
{
    double pl, cl, pr, cr, FL[OR_MAXV], FR[OR_MAXV];
    closure(c, UL, x, y, &pl, &cl);
    closure(c, UR, x, y, &pr, &cr);
    flux_n(c, UL, pl, nx, ny, FL);
    flux_n(c, UR, pr, nx, ny, FR);
    double rl = UL[0], rr = UR[0];
    double ql = (UL[1] * nx + UL[2] * ny) / rl, qr = (UR[1] * nx + UR[2] * ny) / rr;
    double sl = fmin(ql - cl, qr - cr), sr = fmax(ql + cl, qr + cr);
    double ss = (pr - pl + rl * ql * (sl - ql) - rr * qr * (sr - qr)) / (rl * (sl - ql) - rr * (sr - qr));
    if (sl >= 0.0) {
        for (int v = 0; v < 4; ++v) h[v] = FL[v];
        return;
    }
    if (sr <= 0.0) {
        for (int v = 0; v < 4; ++v) h[v] = FR[v];
        return;
    }
    /* the side whose star state the edge sees */
    const int left = ss >= 0.0;
    const double *U = left ? UL : UR, *F = left ? FL : FR;
    double sk = left ? sl : sr, qk = left ? ql : qr, pk = left ? pl : pr, rk = U[0];
    double f = rk * (sk - qk) / (sk - ss);
    double us[4];
    us[0] = f;
    us[1] = f * (U[1] / rk + (ss - qk) * nx);
    us[2] = f * (U[2] / rk + (ss - qk) * ny);
    us[3] = f * (U[3] / rk + (ss - qk) * (ss + pk / (rk * (sk - qk))));
    for (int v = 0; v < 4; ++v) h[v] = F[v] + sk * (us[v] - U[v]);
}

/* the configured numerical flux of eq. (3) */
static void num_flux(const or_cfg *c, const double *Ui, const double *Uo, double nx, double ny, double x, double y,
                     double *h)
{
    if (c->flux == 1 && c->closure == 2)
        hllc(c, Ui, Uo, nx, ny, x, y, h);
    else
        rusanov(c, Ui, Uo, nx, ny, x, y, h);
}

void or_num_flux(const or_cfg *c, const double *Ui, const double *Uo, double nx, double ny, double x, double y,
                 double *h)
{
    num_flux(c, Ui, Uo, nx, ny, x, y, h);
}

/* ------------------------------------------------------------------ */
/* initial projection (Sec. 3.1 (i))                                     */
/* ------------------------------------------------------------------ */

void or_project(const or_cfg *c, const double *prim, double *u)
{
    tables T;
    make_tables(c, &T);
    long E = (long)c->nx * c->ny;
    int n = c->n;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                double s[OR_MAXV] = {0.0, 0.0, 0.0, 0.0};
                for (int q = 0; q < n; ++q)
                    for (int r = 0; r < n; ++r) {
                        long k = q * n + r;
                        double rho = prim[(0 * E + e) * T.nn + k];
                        double vx = prim[(1 * E + e) * T.nn + k];
                        double vy = prim[(2 * E + e) * T.nn + k];
                        double U[OR_MAXV];
                        /* (b) primitive -> conservative */
                        U[0] = rho;
                        U[1] = rho * vx;
                        U[2] = rho * vy;
                        if (c->nvar == 4) {
                            double p = prim[(3 * E + e) * T.nn + k];
                            U[3] = p / (c->gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy);
                        }
                        /* (c) L2 projection by the (n x n) Gauss rule */
                        double wphi = T.wh[q] * T.wh[r] * T.phi[a][q] * T.phi[b][r];
                        for (int v = 0; v < c->nvar; ++v) s[v] += U[v] * wphi;
                    }
                for (int v = 0; v < c->nvar; ++v) u[((long)v * T.nn + a * n + b) * E + e] = s[v];
            }
    }
}

/* ------------------------------------------------------------------ */
/* right-hand side L(u) of eq. (3)                                       */
/* ------------------------------------------------------------------ */

void or_rhs(const or_cfg *c, double t, const double *u, const double *u0, double *rhs)
{
    tables T;
    make_tables(c, &T);
    long E = (long)c->nx * c->ny;
    int n = c->n, nv = c->nvar;
    const double dx = T.dx, dy = T.dy;

#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        int i = (int)(e % c->nx), j = (int)(e / c->nx);
        double xc = elem_xc(c, &T, i), yc = elem_yc(c, &T, j);
        double R[OR_MAXV][OR_MAXN * OR_MAXN];
        memset(R, 0, sizeof R);

        /* volume terms: sum_j [f . grad v + S v] w_j |K| / |K| */
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r) {
                double U[OR_MAXV];
                for (int v = 0; v < nv; ++v) {
                    double s = 0.0;
                    for (int a = 0; a < n; ++a)
                        for (int b = 0; b < n; ++b)
                            s += u[((long)v * T.nn + a * n + b) * E + e] * T.phi[a][q] * T.phi[b][r];
                    U[v] = s;
                }
                double x = xc + 0.5 * dx * T.xi[q], y = yc + 0.5 * dy * T.xi[r];
                double p, cs, fx[OR_MAXV], fy[OR_MAXV], S[OR_MAXV], gx, gy;
                closure(c, U, x, y, &p, &cs);
                flux_n(c, U, p, 1.0, 0.0, fx);
                flux_n(c, U, p, 0.0, 1.0, fy);
                grad_phi(c, x, y, t, &gx, &gy);
                S[0] = 0.0;
                S[1] = -U[0] * gx;
                S[2] = -U[0] * gy;
                if (nv == 4) S[3] = -(U[1] * gx + U[2] * gy);
                double wq = T.wh[q] * T.wh[r];
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) {
                        double dvx = (2.0 / dx) * T.dphi[a][q] * T.phi[b][r]; /* d/dx of phi_ab */
                        double dvy = (2.0 / dy) * T.phi[a][q] * T.dphi[b][r]; /* d/dy of phi_ab */
                        double vv = T.phi[a][q] * T.phi[b][r];
                        for (int v = 0; v < nv; ++v)
                            R[v][a * n + b] += wq * (fx[v] * dvx + fy[v] * dvy + S[v] * vv);
                    }
            }

        /* edge terms: - sum_e sum_i h_{e,K}(x_i) v(x_i) w_i |e| / |K| */
        for (int f = 0; f < 4; ++f) {
            /* f: 0 west (xi=-1), 1 east (xi=+1), 2 south (eta=-1), 3 north (eta=+1) */
            double nx = f == 0 ? -1.0 : (f == 1 ? 1.0 : 0.0);
            double ny = f == 2 ? -1.0 : (f == 3 ? 1.0 : 0.0);
            int in = i + (f == 1) - (f == 0), jn = j + (f == 3) - (f == 2);
            int outside = in < 0 || in >= c->nx || jn < 0 || jn >= c->ny;
            if (in < 0) in += c->nx;
            if (in >= c->nx) in -= c->nx;
            if (jn < 0) jn += c->ny;
            if (jn >= c->ny) jn -= c->ny;
            long en = (long)jn * c->nx + in;
            double len_over_area = (f < 2) ? 1.0 / dx : 1.0 / dy;
            for (int k = 0; k < n; ++k) {
                double xi = f < 2 ? (f == 0 ? -1.0 : 1.0) : T.xi[k];
                double eta = f < 2 ? T.xi[k] : (f == 2 ? -1.0 : 1.0);
                double Ui[OR_MAXV], Uo[OR_MAXV], h[OR_MAXV];
                eval_point(c, u, e, xi, eta, Ui);
                if (outside && c->bc == 1) {
                    /* fixed box edge: exterior state = initial interior trace */
                    eval_point(c, u0, e, xi, eta, Uo);
                } else if (outside && c->bc == 2) {
                    /* gradient-free box edge (Sec. 4.2): a ghost element with no
                     * gradient, the element's own mean state */
                    for (int v = 0; v < nv; ++v) Uo[v] = u[((long)v * T.nn) * E + e];
                } else {
                    /* the same physical point seen from the neighbour */
                    double xin = f < 2 ? -xi : xi, etan = f < 2 ? eta : -eta;
                    eval_point(c, u, en, xin, etan, Uo);
                }
                double x = xc + 0.5 * dx * xi, y = yc + 0.5 * dy * eta;
                num_flux(c, Ui, Uo, nx, ny, x, y, h);
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) {
                        double vv = or_phi(a, xi) * or_phi(b, eta);
                        for (int v = 0; v < nv; ++v) R[v][a * n + b] -= len_over_area * T.wh[k] * h[v] * vv;
                    }
            }
        }
        for (int v = 0; v < nv; ++v)
            for (int m = 0; m < T.nn; ++m) rhs[((long)v * T.nn + m) * E + e] = R[v][m];
    }
}

/* ------------------------------------------------------------------ */
/* CFL time step (Sec. 2.3)                                              */
/* ------------------------------------------------------------------ */

double or_dt(const or_cfg *c, const double *u)
{
    tables T;
    make_tables(c, &T);
    long E = (long)c->nx * c->ny;
    double fac = 1.0 / (2.0 * (c->n - 1) + 1.0);
    if (c->positivity) {
        /* Sec. 2.4: min(1/(2N_p+1), w_1/2), w_1 of the rule normalised to sum 1 */
        double xl[OR_MAXN + 1], wl[OR_MAXN + 1];
        or_gauss_lobatto(or_pp_lobatto_points(c->n - 1), xl, wl);
        double w1 = 0.5 * wl[0];
        if (0.5 * w1 < fac) fac = 0.5 * w1;
    }
    fac *= c->cfl;
    double dtmin = INFINITY;
    for (long e = 0; e < E; ++e) {
        int i = (int)(e % c->nx), j = (int)(e / c->nx);
        double U[OR_MAXV];
        for (int v = 0; v < c->nvar; ++v) U[v] = u[((long)v * T.nn) * E + e]; /* mode 00 = mean */
        double p, cs;
        closure(c, U, elem_xc(c, &T, i), elem_yc(c, &T, j), &p, &cs);
        double sx = (fabs(U[1] / U[0]) + cs) / T.dx;
        double sy = (fabs(U[2] / U[0]) + cs) / T.dy;
        double dtk = fac / (sx + sy);
        if (dtk < dtmin) dtmin = dtk;
    }
    return dtmin;
}

/* ------------------------------------------------------------------ */
/* Runge-Kutta in Butcher form (Algorithm 1, Appendix A)                 */
/* ------------------------------------------------------------------ */

void or_rk_butcher(int s, const double *A, const double *b, const double *cc,
                   or_rhs_fn f, void *ctx, long N, double *u, double t, double dt)
{
    double *k = (double *)malloc(sizeof(double) * (size_t)s * (size_t)N);
    double *y = (double *)malloc(sizeof(double) * (size_t)N);
    for (int i = 0; i < s; ++i) {
        for (long x = 0; x < N; ++x) {
            double acc = 0.0;
            for (int jj = 0; jj < i; ++jj) acc += A[i * s + jj] * k[(long)jj * N + x];
            y[x] = u[x] + dt * acc;
        }
        f(ctx, t + cc[i] * dt, y, k + (long)i * N);
    }
    for (long x = 0; x < N; ++x) {
        double acc = 0.0;
        for (int i = 0; i < s; ++i) acc += b[i] * k[(long)i * N + x];
        u[x] += dt * acc;
    }
    free(k);
    free(y);
}

/* SSP(3,3): the printed table has c_3 = 3/4 next to a_31 + a_32 = 1/2; the
 * row-sum condition c_i = sum_j a_ij fixes c_3 = 1/2. */
void or_ssprk3_tableau(double *A, double *b, double *cc)
{
    for (int i = 0; i < 9; ++i) A[i] = 0.0;
    A[1 * 3 + 0] = 1.0;
    A[2 * 3 + 0] = 0.25;
    A[2 * 3 + 1] = 0.25;
    b[0] = 1.0 / 6.0;
    b[1] = 1.0 / 6.0;
    b[2] = 2.0 / 3.0;
    cc[0] = 0.0;
    cc[1] = 1.0;
    cc[2] = 0.5;
}

typedef struct {
    const or_cfg *c;
    const double *u0;
} dg_ctx;

static void dg_rhs_cb(void *ctx, double t, const double *u, double *k)
{
    dg_ctx *d = (dg_ctx *)ctx;
    or_rhs(d->c, t, u, d->u0, k);
}

/* The other tables of Appendix A.  SSP(2,2) is printed with a_21 = c_2 = 1/2
 * and b = (1/2, 1/2), which is first order only (b.c = 1/4); the two-stage
 * SSP scheme of order two is Heun's, a_21 = c_2 = 1.  The five-stage table
 * (captioned RK(4,5): fourth order, five stages) and the Cash-Karp table are
 * taken as printed; Cash-Karp advances with its fifth-order weights. */
int or_rk_tableau(int kind, double *A, double *b, double *cc)
{
    for (int i = 0; i < 36; ++i) A[i] = 0.0;
    for (int i = 0; i < 6; ++i) b[i] = cc[i] = 0.0;
    if (kind == 0) {
        double A3[9];
        or_ssprk3_tableau(A3, b, cc);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A[i * 6 + j] = A3[i * 3 + j];
        return 3;
    }
    if (kind == 1) {
        A[1 * 6 + 0] = 1.0;
        b[0] = 0.5;
        b[1] = 0.5;
        cc[1] = 1.0;
        return 2;
    }
    if (kind == 2) {
        static const double a[5][4] = {
            {0.0, 0.0, 0.0, 0.0},
            {0.39175222700392, 0.0, 0.0, 0.0},
            {0.21766909633821, 0.36841059262959, 0.0, 0.0},
            {0.08269208670950, 0.13995850206999, 0.25189177424738, 0.0},
            {0.06796628370320, 0.11503469844438, 0.20703489864929, 0.54497475021237}};
        static const double bb[5] = {0.14681187618661, 0.24848290924556, 0.10425883036650,
                                     0.27443890091960, 0.22600748319395};
        static const double c5[5] = {0.0, 0.39175222700392, 0.58607968896779, 0.47454236302687,
                                     0.93501063100924};
        for (int i = 0; i < 5; ++i) {
            for (int j = 0; j < 4; ++j) A[i * 6 + j] = a[i][j];
            b[i] = bb[i];
            cc[i] = c5[i];
        }
        return 5;
    }
    if (kind == 3) {
        A[1 * 6 + 0] = 1.0 / 5.0;
        A[2 * 6 + 0] = 3.0 / 40.0;
        A[2 * 6 + 1] = 9.0 / 40.0;
        A[3 * 6 + 0] = 3.0 / 10.0;
        A[3 * 6 + 1] = -9.0 / 10.0;
        A[3 * 6 + 2] = 6.0 / 5.0;
        A[4 * 6 + 0] = -11.0 / 54.0;
        A[4 * 6 + 1] = 5.0 / 2.0;
        A[4 * 6 + 2] = -70.0 / 27.0;
        A[4 * 6 + 3] = 35.0 / 27.0;
        A[5 * 6 + 0] = 1631.0 / 55296.0;
        A[5 * 6 + 1] = 175.0 / 512.0;
        A[5 * 6 + 2] = 575.0 / 13824.0;
        A[5 * 6 + 3] = 44275.0 / 110592.0;
        A[5 * 6 + 4] = 253.0 / 4096.0;
        b[0] = 37.0 / 378.0;
        b[2] = 250.0 / 621.0;
        b[3] = 125.0 / 594.0;
        b[5] = 512.0 / 1771.0;
        cc[1] = 1.0 / 5.0;
        cc[2] = 3.0 / 10.0;
        cc[3] = 3.0 / 5.0;
        cc[4] = 1.0;
        cc[5] = 7.0 / 8.0;
        return 6;
    }
    return -1;
}

double or_step(const or_cfg *c, double *u, double t, double dt_fixed, const double *u0)
{
    double A6[36], b6[6], c6[6];
    int s = or_rk_tableau(c->rk, A6, b6, c6);
    if (s < 0) return -1.0;
    double A[36];
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) A[i * s + j] = A6[i * 6 + j];
    double dt = dt_fixed > 0.0 ? dt_fixed : or_dt(c, u);
    dg_ctx d = {c, u0};
    long N = (long)c->nvar * c->n * c->n * c->nx * c->ny;
    or_rk_butcher(s, A, b6, c6, dg_rhs_cb, &d, N, u, t, dt);
    if (c->damping) or_damp(c, u, u0, dt);
    return dt;
}

/* ------------------------------------------------------------------ */
/* wave-killing damping (Sec. 5.1)                                       */
/* ------------------------------------------------------------------ */

/* ramp R(r) and the damping radius of its zone: R = ((r - r_d)/(r_b - r_d))^2
 * between the damping radius r_d (R = 0) and the boundary radius r_b (R = 1),
 * with r_b = r_d / 1.15^(3/2) inside and r_d * 1.15^(3/2) outside; clamped
 * to [0, 1]. */
static double ramp(const or_cfg *c, double r, double *rd)
{
    double f = pow(1.15, 1.5);
    if (r < c->rd_in) {
        double rb = c->rd_in / f;
        double s = (r - c->rd_in) / (rb - c->rd_in);
        *rd = c->rd_in;
        return s > 1.0 ? 1.0 : s * s;
    }
    if (r > c->rd_out) {
        double rb = c->rd_out * f;
        double s = (r - c->rd_out) / (rb - c->rd_out);
        *rd = c->rd_out;
        return s > 1.0 ? 1.0 : s * s;
    }
    *rd = c->rd_in;
    return 0.0;
}

/* Q <- (dt Q0 + tau Q) / (tau + dt) with tau = 2 pi sqrt(r_d^3/GM) / R(r),
 * written as Q + w (Q0 - Q), w = dt R / (T_d + dt R), for Q = rho, v (and the
 * temperature p/rho when adiabatic) at the volume nodes; the nodal increment
 * of the conservative variables is projected and added to the modes. */
void or_damp(const or_cfg *c, double *u, const double *u0, double dt)
{
    tables T;
    make_tables(c, &T);
    long E = (long)c->nx * c->ny;
    int n = c->n, nv = c->nvar;
    const double pi = 3.14159265358979323846;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        int i = (int)(e % c->nx), j = (int)(e / c->nx);
        double xc = elem_xc(c, &T, i), yc = elem_yc(c, &T, j);
        double D[OR_MAXV][OR_MAXN * OR_MAXN];
        int any = 0;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r) {
                double x = xc + 0.5 * T.dx * T.xi[q], y = yc + 0.5 * T.dy * T.xi[r];
                double rd, R = ramp(c, sqrt(x * x + y * y), &rd);
                for (int v = 0; v < nv; ++v) D[v][q * n + r] = 0.0;
                if (R <= 0.0) continue;
                any = 1;
                double U[OR_MAXV], U0[OR_MAXV];
                for (int v = 0; v < nv; ++v) {
                    double s = 0.0, s0 = 0.0;
                    for (int a = 0; a < n; ++a)
                        for (int b = 0; b < n; ++b) {
                            long idx = ((long)v * T.nn + a * n + b) * E + e;
                            s += u[idx] * T.phi[a][q] * T.phi[b][r];
                            s0 += u0[idx] * T.phi[a][q] * T.phi[b][r];
                        }
                    U[v] = s;
                    U0[v] = s0;
                }
                double Td = 2.0 * pi * sqrt(rd * rd * rd / c->gm);
                double w = dt * R / (Td + dt * R);
                double rho = U[0], vx = U[1] / U[0], vy = U[2] / U[0];
                double rho0 = U0[0], vx0 = U0[1] / U0[0], vy0 = U0[2] / U0[0];
                double drho = w * (rho0 - rho);
                double dvx = w * (vx0 - vx), dvy = w * (vy0 - vy);
                double rho1 = rho + drho, vx1 = vx + dvx, vy1 = vy + dvy;
                D[0][q * n + r] = drho;
                D[1][q * n + r] = rho * dvx + drho * vx1;
                D[2][q * n + r] = rho * dvy + drho * vy1;
                if (nv == 4) {
                    double ke = 0.5 * rho * (vx * vx + vy * vy);
                    double T1 = (c->gamma - 1.0) * (U[3] - ke) / rho;
                    double ke0 = 0.5 * rho0 * (vx0 * vx0 + vy0 * vy0);
                    double T0 = (c->gamma - 1.0) * (U0[3] - ke0) / rho0;
                    double dT = w * (T0 - T1);
                    double dp = rho * dT + drho * (T1 + dT);
                    /* rho1 |v1|^2 - rho |v|^2 = drho |v1|^2 + rho (v1 - v).(v1 + v) */
                    double dke = 0.5 * (drho * (vx1 * vx1 + vy1 * vy1) +
                                        rho * (dvx * (vx1 + vx) + dvy * (vy1 + vy)));
                    D[3][q * n + r] = dp / (c->gamma - 1.0) + dke;
                }
            }
        if (!any) continue;
        for (int v = 0; v < nv; ++v)
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    double s = 0.0;
                    for (int q = 0; q < n; ++q)
                        for (int r = 0; r < n; ++r)
                            s += T.wh[q] * T.wh[r] * D[v][q * n + r] * T.phi[a][q] * T.phi[b][r];
                    u[((long)v * T.nn + a * n + b) * E + e] += s;
                }
    }
}

/* ------------------------------------------------------------------ */
/* torque on the planet (Sec. 5.2, eq. (5))                              */
/* ------------------------------------------------------------------ */

/* Gamma_z = r_p x sum_n M_n (r_n - r_p) / (|r_n - r_p|^2 + eps^2)^(3/2), G = 1,
 * with the cells read as the volume Gauss nodes of every element carrying the
 * mass rho_h(x_qr) w_q w_r |K| / 4. */
double or_torque(const or_cfg *c, double t, const double *u, double *sum_abs)
{
    tables T;
    make_tables(c, &T);
    long E = (long)c->nx * c->ny;
    int n = c->n;
    double xp, yp;
    or_planet_pos(c, t, &xp, &yp);
    double area = T.dx * T.dy;
    double tot = 0.0, tabs = 0.0;
    for (long e = 0; e < E; ++e) {
        int i = (int)(e % c->nx), j = (int)(e / c->nx);
        double xc = elem_xc(c, &T, i), yc = elem_yc(c, &T, j);
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r) {
                double rho = 0.0;
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) rho += u[((long)a * n + b) * E + e] * T.phi[a][q] * T.phi[b][r];
                double x = xc + 0.5 * T.dx * T.xi[q], y = yc + 0.5 * T.dy * T.xi[r];
                double m = rho * T.wh[q] * T.wh[r] * area;
                double dx = x - xp, dy = y - yp;
                double d2 = dx * dx + dy * dy + c->eps * c->eps;
                double k = m / (d2 * sqrt(d2));
                double term = xp * (k * dy) - yp * (k * dx);
                tot += term;
                tabs += fabs(term);
            }
    }
    if (sum_abs) *sum_abs = tabs;
    return tot;
}
