/*
 * Troubled-cell treatment for the plain FP64 CPU oracle: the modal-decay
 * indicator, the Cockburn-Shu minmod limiter (the DG formulation the paper
 * follows, Sec. 2.2), the limited SSP-RK3 step, and the small learned
 * indicator (MLP) with its loss gradient and the Adam update.
 *
 * TEST INFRASTRUCTURE ONLY -- see dg_oracle.h.  Plain loops in FP64; the
 * MLP's bfloat16 operand rounding is emulated where asked.
 */
#include "dg_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void or_indicator(const or_cfg *c, const double *u, double *s)
{
    long E = (long)c->nx * c->ny;
    int n = c->n, p = c->n - 1;
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        double top = 0.0, all = 0.0;
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                double v = u[((long)a * n + b) * E + e];
                all += v * v;
                if (a == p || b == p) top += v * v;
            }
        s[e] = (all > 0.0 && top > 0.0) ? log10(top / all) : -300.0;
    }
}

static double minmod3(double a, double b, double c)
{
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}

/* mean of variable v of the neighbour across edge f (0 W, 1 E, 2 S, 3 N) */
static double nb_mean(const or_cfg *c, const double *u, const double *u0, long e, int v, int f)
{
    long E = (long)c->nx * c->ny;
    int nn = c->n * c->n;
    int i = (int)(e % c->nx), j = (int)(e / c->nx);
    int in = i + (f == 1) - (f == 0), jn = j + (f == 3) - (f == 2);
    int outside = in < 0 || in >= c->nx || jn < 0 || jn >= c->ny;
    if (outside && c->bc == 1) return u0[((long)v * nn) * E + e];
    if (outside && c->bc == 2) return u[((long)v * nn) * E + e]; /* gradient-free: own mean */
    in = (in + c->nx) % c->nx;
    jn = (jn + c->ny) % c->ny;
    return u[((long)v * nn) * E + (long)jn * c->nx + in];
}

void or_minmod(const or_cfg *c, double *u, const double *u0, const unsigned char *flag,
               unsigned char *changed)
{
    long E = (long)c->nx * c->ny;
    int n = c->n, nn = n * n, nv = c->nvar;
    const double r3 = sqrt(3.0);
    /* means are never modified, so neighbours may be read from u in place */
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        changed[e] = 0;
        if (!flag[e]) continue;
        double sx[4], sy[4];
        int any = 0;
        for (int v = 0; v < nv; ++v) {
            double m = u[((long)v * nn) * E + e];
            double ax = r3 * u[((long)v * nn + 1 * n + 0) * E + e]; /* mode (1,0): edge jump in x */
            double ay = r3 * u[((long)v * nn + 0 * n + 1) * E + e]; /* mode (0,1): edge jump in y */
            double lx = minmod3(ax, nb_mean(c, u, u0, e, v, 1) - m, m - nb_mean(c, u, u0, e, v, 0));
            double ly = minmod3(ay, nb_mean(c, u, u0, e, v, 3) - m, m - nb_mean(c, u, u0, e, v, 2));
            sx[v] = lx;
            sy[v] = ly;
            if (lx != ax || ly != ay) any = 1;
        }
        if (!any) continue;
        changed[e] = 1;
        for (int v = 0; v < nv; ++v)
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    long idx = ((long)v * nn + a * n + b) * E + e;
                    if (a == 0 && b == 0) continue;
                    if (a == 1 && b == 0)
                        u[idx] = sx[v] / r3;
                    else if (a == 0 && b == 1)
                        u[idx] = sy[v] / r3;
                    else
                        u[idx] = 0.0;
                }
    }
}

/* ------------------------------------------------------------------ */
/* positivity-preserving limiter (Sec. 2.4; Zhang & Shu 2010)            */
/* ------------------------------------------------------------------ */

#define PP_MAXP 16 /* points per direction of either rule, generous */

/* value of variable v of element e at reference point (xi, eta) */
static double point_value(const or_cfg *c, const double *u, long e, int v, double xi, double eta)
{
    long E = (long)c->nx * c->ny;
    int n = c->n;
    double s = 0.0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) s += u[((long)v * n * n + a * n + b) * E + e] * or_phi(a, xi) * or_phi(b, eta);
    return s;
}

static double pressure_of(const or_cfg *c, const double *U)
{
    return (c->gamma - 1.0) * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0]);
}

void or_positivity(const or_cfg *c, double *u, unsigned char *changed, double *theta)
{
    long E = (long)c->nx * c->ny;
    int n = c->n, nn = n * n, nv = c->nvar;
    const int adi = c->closure == 2;
    /* the test points: (Lobatto x Gauss) and (Gauss x Lobatto) */
    double xg[PP_MAXP], wg[PP_MAXP], xl[PP_MAXP], wl[PP_MAXP];
    or_gauss_legendre(n, xg, wg);
    int L = or_pp_lobatto_points(n - 1);
    or_gauss_lobatto(L, xl, wl);
    int np = 2 * L * n;
    double *px = (double *)malloc(sizeof(double) * np), *py = (double *)malloc(sizeof(double) * np);
    int k = 0;
    for (int q = 0; q < L; ++q)
        for (int r = 0; r < n; ++r) {
            px[k] = xl[q];
            py[k] = xg[r];
            ++k;
        }
    for (int q = 0; q < n; ++q)
        for (int r = 0; r < L; ++r) {
            px[k] = xg[q];
            py[k] = xl[r];
            ++k;
        }
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        double M[4];
        for (int v = 0; v < nv; ++v) M[v] = u[((long)v * nn) * E + e];
        double th1 = 1.0, th2 = 1.0;
        changed[e] = 0;
        double pbar = adi ? pressure_of(c, M) : M[0];
        if (!(M[0] > 0.0) || !(pbar > 0.0)) {
            if (theta) theta[2 * e] = theta[2 * e + 1] = 1.0;
            continue;
        }
        double eps = c->pp_eps > 0.0 ? c->pp_eps : 1e-13;
        if (M[0] < eps) eps = M[0];
        if (adi && pbar < eps) eps = pbar;
        /* density */
        double rmin = INFINITY;
        for (int k2 = 0; k2 < np; ++k2) {
            double r = point_value(c, u, e, 0, px[k2], py[k2]);
            if (r < rmin) rmin = r;
        }
        if (rmin < eps) {
            th1 = (M[0] - eps) / (M[0] - rmin);
            for (int m = 1; m < nn; ++m) u[((long)m) * E + e] *= th1;
        }
        /* pressure, with the density already limited */
        if (adi) {
            for (int k2 = 0; k2 < np; ++k2) {
                double W[4];
                for (int v = 0; v < 4; ++v) W[v] = point_value(c, u, e, v, px[k2], py[k2]);
                if (!(pressure_of(c, W) < eps)) continue;
                /* p(M + t (W - M)) is concave in t, >= eps at 0 and < eps at 1:
                 * the admissible t form [0, t*].  Bisection on the condition
                 * p >= eps itself, keeping the admissible end (the
                 * closed-form root of the equivalent quadratic loses digits
                 * near a double root, and a point left at p < 0 breaks the
                 * sound speed). */
                double lo = 0.0, hi = 1.0;
                for (int it = 0; it < 64; ++it) {
                    double mid = 0.5 * (lo + hi), S[4];
                    for (int v = 0; v < 4; ++v) S[v] = M[v] + mid * (W[v] - M[v]);
                    if (pressure_of(c, S) >= eps)
                        lo = mid;
                    else
                        hi = mid;
                }
                if (lo < th2) th2 = lo;
            }
            if (th2 < 1.0)
                for (int v = 0; v < nv; ++v)
                    for (int m = 1; m < nn; ++m) u[((long)v * nn + m) * E + e] *= th2;
        }
        if (theta) {
            theta[2 * e] = th1;
            theta[2 * e + 1] = th2;
        }
        changed[e] = th1 < 1.0 || th2 < 1.0;
    }
    free(px);
    free(py);
}

static void limit_state(const or_cfg *c, double *u, const double *u0, double s0)
{
    long E = (long)c->nx * c->ny;
    double *s = (double *)malloc(sizeof(double) * E);
    unsigned char *fl = (unsigned char *)malloc(E), *ch = (unsigned char *)malloc(E);
    or_indicator(c, u, s);
    for (long e = 0; e < E; ++e) fl[e] = s[e] > s0;
    or_minmod(c, u, u0, fl, ch);
    if (c->positivity) or_positivity(c, u, ch, NULL);
    free(s);
    free(fl);
    free(ch);
}

/* u1 = Lim(u + dt L(u)); u2 = Lim(3/4 u + 1/4 (u1 + dt L(u1))); u3 = Lim(1/3 u + 2/3 (u2 + dt L(u2)));
 * stage times t, t + dt, t + dt/2; then damping */
double or_step_limited(const or_cfg *c, double *u, double t, double dt_fixed, const double *u0, double s0)
{
    long N = (long)c->nvar * c->n * c->n * c->nx * c->ny;
    double dt = dt_fixed > 0.0 ? dt_fixed : or_dt(c, u);
    double *k = (double *)malloc(sizeof(double) * N);
    double *u1 = (double *)malloc(sizeof(double) * N);
    double *u2 = (double *)malloc(sizeof(double) * N);
    or_rhs(c, t, u, u0, k);
    for (long x = 0; x < N; ++x) u1[x] = u[x] + dt * k[x];
    limit_state(c, u1, u0, s0);
    or_rhs(c, t + dt, u1, u0, k);
    for (long x = 0; x < N; ++x) u2[x] = 0.75 * u[x] + 0.25 * (u1[x] + dt * k[x]);
    limit_state(c, u2, u0, s0);
    or_rhs(c, t + 0.5 * dt, u2, u0, k);
    for (long x = 0; x < N; ++x) u[x] = u[x] / 3.0 + 2.0 / 3.0 * (u2[x] + dt * k[x]);
    limit_state(c, u, u0, s0);
    if (c->damping) {
        or_damp(c, u, u0, dt);
        /* the damping changes the state once more: positivity again */
        if (c->positivity) {
            unsigned char *ch = (unsigned char *)malloc((size_t)c->nx * c->ny);
            or_positivity(c, u, ch, NULL);
            free(ch);
        }
    }
    free(k);
    free(u1);
    free(u2);
    return dt;
}

/* ------------------------------------------------------------------ MLP */

void or_mlp_features(const or_cfg *c, const double *u, const double *scale, double *f)
{
    long E = (long)c->nx * c->ny;
    int nn = c->n * c->n, nv = c->nvar;
    for (long e = 0; e < E; ++e)
        for (int v = 0; v < nv; ++v) {
            double d = fabs(u[((long)v * nn) * E + e]) + scale[v];
            for (int m = 0; m < nn; ++m) f[e * (nv * nn) + v * nn + m] = u[((long)v * nn + m) * E + e] / d;
        }
}

double or_bf16(double x)
{
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return x; /* inf / nan */
    b += 0x7fffu + ((b >> 16) & 1u);
    b &= 0xffff0000u;
    memcpy(&f, &b, 4);
    return (double)f;
}

#define MLP_IN 64
#define MLP_H 32
/* parameter offsets */
#define P_W1 0
#define P_B1 (P_W1 + MLP_H * MLP_IN)
#define P_W2 (P_B1 + MLP_H)
#define P_B2 (P_W2 + MLP_H * MLP_H)
#define P_W3 (P_B2 + MLP_H)
#define P_B3 (P_W3 + MLP_H)

static double rb(double x, int bf16) { return bf16 ? or_bf16(x) : x; }
static double rf(double x, int bf16) { return bf16 ? (double)(float)x : x; }

/* one sample: returns the logit; fills the activations fed forward (a1, a2)
 * and the pre-activations (z1, z2) */
static double fwd1(const double *par, const double *x, int bf16, double *a1, double *a2, double *z1,
                   double *z2)
{
    double xin[MLP_IN];
    for (int k = 0; k < MLP_IN; ++k) xin[k] = rb(x[k], bf16);
    for (int o = 0; o < MLP_H; ++o) {
        double s = 0.0;
        for (int k = 0; k < MLP_IN; ++k) s += rb(par[P_W1 + o * MLP_IN + k], bf16) * xin[k];
        z1[o] = rf(s, bf16) + par[P_B1 + o];
        a1[o] = rb(z1[o] > 0.0 ? z1[o] : 0.0, bf16);
    }
    for (int o = 0; o < MLP_H; ++o) {
        double s = 0.0;
        for (int k = 0; k < MLP_H; ++k) s += rb(par[P_W2 + o * MLP_H + k], bf16) * a1[k];
        z2[o] = rf(s, bf16) + par[P_B2 + o];
        a2[o] = rb(z2[o] > 0.0 ? z2[o] : 0.0, bf16);
    }
    double s = 0.0;
    for (int k = 0; k < MLP_H; ++k) s += rb(par[P_W3 + k], bf16) * a2[k];
    return rf(s, bf16) + par[P_B3];
}

void or_mlp_forward(const double *par, const double *x, long nb, int bf16, double *z, double *h1,
                    double *h2)
{
    for (long i = 0; i < nb; ++i) {
        double a1[MLP_H], a2[MLP_H], z1[MLP_H], z2[MLP_H];
        z[i] = fwd1(par, x + i * MLP_IN, bf16, a1, a2, z1, z2);
        if (h1) memcpy(h1 + i * MLP_H, a1, sizeof a1);
        if (h2) memcpy(h2 + i * MLP_H, a2, sizeof a2);
    }
}

/* loss = mean_i [ -w_i ( y_i log s(z_i) + (1 - y_i) log(1 - s(z_i)) ) ], w_i = pos_weight for y=1;
 * dloss/dz_i = ( pos_weight y_i (s - 1) + (1 - y_i) s ) / nb */
double or_mlp_loss_grad(const double *par, const double *x, const double *y, long nb, double pos_weight,
                        int bf16, double *grad)
{
    memset(grad, 0, sizeof(double) * OR_MLP_NPARAM);
    double loss = 0.0;
    for (long i = 0; i < nb; ++i) {
        double xin[MLP_IN], a1[MLP_H], a2[MLP_H], z1[MLP_H], z2[MLP_H];
        double z = fwd1(par, x + i * MLP_IN, bf16, a1, a2, z1, z2);
        for (int k = 0; k < MLP_IN; ++k) xin[k] = rb(x[i * MLP_IN + k], bf16);
        /* log s(z) = -log(1 + e^-z), log(1 - s(z)) = -log(1 + e^z), stably */
        double lsp = z >= 0 ? -log1p(exp(-z)) : z - log1p(exp(z));
        double lsn = z >= 0 ? -z - log1p(exp(-z)) : -log1p(exp(z));
        double sg = 1.0 / (1.0 + exp(-z));
        loss += -(pos_weight * y[i] * lsp + (1.0 - y[i]) * lsn);
        double dz = (pos_weight * y[i] * (sg - 1.0) + (1.0 - y[i]) * sg) / nb;
        /* output layer */
        grad[P_B3] += dz;
        double d2[MLP_H];
        for (int k = 0; k < MLP_H; ++k) {
            grad[P_W3 + k] += dz * a2[k];
            d2[k] = z2[k] > 0.0 ? dz * rb(par[P_W3 + k], bf16) : 0.0;
        }
        /* hidden layer 2 */
        double d1[MLP_H];
        for (int k = 0; k < MLP_H; ++k) d1[k] = 0.0;
        for (int o = 0; o < MLP_H; ++o) {
            grad[P_B2 + o] += d2[o];
            for (int k = 0; k < MLP_H; ++k) {
                grad[P_W2 + o * MLP_H + k] += d2[o] * a1[k];
                d1[k] += d2[o] * rb(par[P_W2 + o * MLP_H + k], bf16);
            }
        }
        /* hidden layer 1 */
        for (int o = 0; o < MLP_H; ++o) {
            double g1 = z1[o] > 0.0 ? d1[o] : 0.0;
            grad[P_B1 + o] += g1;
            for (int k = 0; k < MLP_IN; ++k) grad[P_W1 + o * MLP_IN + k] += g1 * xin[k];
        }
    }
    return loss / nb;
}

void or_adam(double *par, const double *grad, double *m, double *v, long n, long t, double lr, double b1,
             double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (long k = 0; k < n; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * grad[k];
        v[k] = b2 * v[k] + (1.0 - b2) * grad[k] * grad[k];
        par[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
    }
}
