/*
 * Plain FP64 CPU oracle for the 2D modal discontinuous Galerkin scheme of
 * Velasco Romero, Han Veiga, Teyssier & Masset (2018), "Planet-disc
 * interactions with Discontinuous Galerkin Methods using GPUs".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this library; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library: quadrature, basis, fluxes, time stepping and reductions are all
 * written out again here, as plainly as possible, for checking by eye against
 * the paper.
 *
 * Conventions (own to the oracle, mirrored by its Python wrapper):
 *   n        points per direction = polynomial degree N_p + 1
 *   mode     (a, b), a = degree in x, b = degree in y, flat index a*n + b
 *   node     (q, r), Gauss-Legendre point q in x, r in y, flat index q*n + r
 *   element  e = j*nx + i
 *   state    u[(v*n*n + mode)*E + e]         (one nx*ny plane per mode)
 *   nodes    x[e*n*n + node], y[e*n*n + node]
 *   prim     prim[(v*E + e)*n*n + node]       (rho, vx, vy[, p])
 */
#ifndef DG_ORACLE_H
#define DG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n;            /* points per direction (order m of the scheme) */
    int nvar;         /* 3 (isothermal closures) or 4 (adiabatic) */
    int nx, ny;       /* elements per direction */
    double x0, x1, y0, y1;
    int closure;      /* 0 isothermal c_s, 1 locally isothermal, 2 adiabatic */
    double cs;        /* isothermal sound speed */
    double h;         /* aspect ratio: c_s^2 = h^2 GM / max(r, r_core) */
    double gamma;     /* adiabatic index */
    int bc;           /* 0 periodic, 1 exterior trace = initial trace, 2 gradient-free
                         (exterior state = the element's own current mean) */
    int star;         /* 1: stellar potential (harmonic core inside r_core) */
    double gm, r_core;
    double q, eps;    /* planet mass ratio (0: no planet) and softening */
    double rp, phi0;  /* planet orbit radius and phase at t = 0 */
    int damping;      /* 1: wave-killing zones */
    double rd_in, rd_out;
    double cfl;
    int rk;           /* Appendix A table: 0 SSP(3,3), 1 SSP(2,2), 2 SSP(5,4), 3 Cash-Karp */
    int positivity;   /* 1: positivity-preserving limiter after every stage (Sec. 2.4) */
    double pp_eps;    /* floor of the limiter's eps (<= 0: 1e-13) */
    int flux;         /* edge flux: 0 Rusanov, 1 HLLC (adiabatic closure only) */
} or_cfg;

/* The numerical flux of eq. (3) through an edge point (x, y) with unit
 * outward normal (nx, ny): h(U_in, U_out) of the configured type (c->flux).
 * Exported for its pins. */
void or_num_flux(const or_cfg *c, const double *Ui, const double *Uo, double nx, double ny, double x, double y,
                 double *h);

/* Sec. 2.2, eq. (3): Gauss-Legendre nodes (ascending) and weights on [-1,1]. */
int or_gauss_legendre(int n, double *x, double *w);
/* Gauss-Lobatto nodes (ascending, both ends included) and weights on [-1,1],
 * L >= 2 points: the interior nodes are the roots of P'_{L-1}, the weights
 * 2 / (L (L-1) P_{L-1}(x)^2). */
int or_gauss_lobatto(int L, double *x, double *w);
/* Sec. 2.4: the Gauss-Lobatto rule of the positivity limiter for degree N_p
 * has the fewest points L with 2L - 3 >= N_p */
int or_pp_lobatto_points(int np);
/* Sec. 2.2: orthonormal Legendre basis phi_a = sqrt(2a+1) P_a and derivative. */
double or_phi(int a, double x);
double or_dphi(int a, double x);

/* volume node coordinates of every element */
void or_nodes(const or_cfg *c, double *x, double *y);
/* Sec. 3.1 steps (i)(a)-(c): primitive nodes -> conservative nodes -> modes */
void or_project(const or_cfg *c, const double *prim, double *u);
/* evaluate the modal state at the volume nodes, out[(v*E+e)*n*n + node] */
void or_eval_nodes(const or_cfg *c, const double *u, double *out);
/* eq. (3): du/dt = L(u) at time t.  u0 (initial modes) supplies the exterior
 * traces when bc == 1 and may be NULL for periodic boxes. */
void or_rhs(const or_cfg *c, double t, const double *u, const double *u0, double *rhs);
/* Sec. 2.3: global CFL time step from the element means; with c->positivity
 * the factor C/(2N_p+1) becomes C min(1/(2N_p+1), w_1/2), w_1 the end weight
 * of the limiter's Gauss-Lobatto rule normalised to sum 1 (Sec. 2.4) */
double or_dt(const or_cfg *c, const double *u);

/* Algorithm 1 / Appendix A in Butcher form for a generic right-hand side */
typedef void (*or_rhs_fn)(void *ctx, double t, const double *u, double *k);
void or_rk_butcher(int s, const double *A, const double *b, const double *cc,
                   or_rhs_fn f, void *ctx, long N, double *u, double t, double dt);
/* SSP(3,3) tableau with c = (0, 1, 1/2) */
void or_ssprk3_tableau(double *A9, double *b3, double *c3);
/* Appendix A tables, A row-major s x s in a 6 x 6 array: kind 0 SSP(3,3)
 * (c_3 = 1/2), 1 SSP(2,2) read as Heun (a_21 = c_2 = 1), 2 the five-stage
 * fourth-order SSP table as printed, 3 Cash-Karp with its fifth-order
 * weights.  Returns the number of stages s, or -1 for an unknown kind. */
int or_rk_tableau(int kind, double *A36, double *b6, double *c6);
/* one DG step: dt (CFL if dt_fixed <= 0), the RK stages of c->rk, damping;
 * returns dt (-1 for an unknown c->rk) */
double or_step(const or_cfg *c, double *u, double t, double dt_fixed, const double *u0);

/* Sec. 5.1: wave-killing damping of rho, v (and T) towards the initial state */
void or_damp(const or_cfg *c, double *u, const double *u0, double dt);
/* Sec. 5.2 eq. (5): z-torque of the disc on the planet (G = 1, per unit planet
 * mass); *sum_abs receives the sum of |terms| */
double or_torque(const or_cfg *c, double t, const double *u, double *sum_abs);

/* planet position at time t */
void or_planet_pos(const or_cfg *c, double t, double *xp, double *yp);

/* ---- troubled cells: plain indicator, minmod limiter, learned indicator ---- */

/* modal-decay smoothness of the density of every element:
 * s[e] = log10( sum_{max(a,b) = N_p} u_ab^2 / sum_ab u_ab^2 ) (Parseval, the
 * basis is orthonormal); -300 for an all-zero element */
void or_indicator(const or_cfg *c, const double *u, double *s);
/* Cockburn-Shu TVD minmod limiter on the linear modes of the flagged elements
 * (flag[e] != 0), component-wise on the conservative variables, with the
 * neighbour means (exterior mean = own initial mean at a fixed box edge, from
 * u0).  An element whose slopes change in any variable keeps its means, takes
 * the limited slopes and drops every other mode; changed[e] = 1 then. */
void or_minmod(const or_cfg *c, double *u, const double *u0, const unsigned char *flag,
               unsigned char *changed);
/* Sec. 2.4: positivity-preserving limiter of Zhang & Shu (2010) on every
 * element, in place.  The test points of element K are the tensor sets
 * (Gauss-Lobatto in x) x (Gauss in y) and (Gauss in x) x (Gauss-Lobatto in
 * y), Gauss-Lobatto of or_pp_lobatto_points(N_p) points.  With
 * eps = min(e0, mean density, pressure of the means), e0 = c->pp_eps, or
 * 1e-13 (Zhang & Shu's value) when that is <= 0:
 *   density:  theta1 = min(1, (mean - eps) / (mean - min over the points)),
 *             the density's non-mean modes scaled by theta1;
 *   pressure (adiabatic closure only): at every point where the
 *             pressure of (density-limited) state w is below eps, the largest
 *             t in [0, 1] with p(mean + t (w - mean)) >= eps (64 bisection
 *             steps, keeping the admissible end); theta2 = min of those t
 *             (1 if none); every variable's non-mean modes scaled by theta2.
 * The isothermal closures have p proportional to the density, so the density
 * step covers them.  Elements whose means are not admissible (mean density
 * or pressure <= 0) are left as they are.  changed[e] = 1 where a mode
 * changed; theta (may be NULL) receives theta1, theta2 per element. */
void or_positivity(const or_cfg *c, double *u, unsigned char *changed, double *theta);
/* one SSP-RK3 step in Shu-Osher form with the limiter after every stage:
 * the minmod limiter on the elements with indicator > s0 (s0 = +inf: none),
 * then, if c->positivity, or_positivity; then the damping (if configured),
 * followed by or_positivity once more; returns dt (with c->positivity the
 * CFL factor is C min(1/(2N_p+1), w_1/2), see or_dt) */
double or_step_limited(const or_cfg *c, double *u, double t, double dt_fixed, const double *u0,
                       double s0);

/* learned indicator: 64 -> 32 -> 32 -> 1 MLP, ReLU hidden, sigmoid output.
 * Parameters (FP32 master values held as doubles), flat:
 * W1[32][64], b1[32], W2[32][32], b2[32], w3[32], b3[1]  (3169 values). */
#define OR_MLP_NPARAM 3169
/* features f[e][v*n*n + m] = u_vm / (|u_v00| + scale[v]) */
void or_mlp_features(const or_cfg *c, const double *u, const double *scale, double *f);
/* round to the nearest bfloat16 (ties to even), returned as a double */
double or_bf16(double x);
/* forward pass of nb samples x[nb][64]: with bf16 != 0 the weights, inputs
 * and hidden activations are rounded to bfloat16 before each product and the
 * pre-activations to float32 (the kernel's precision) before rounding; z
 * receives the logits.  h1, h2 (nb x 32, may be NULL) receive the hidden
 * activations as fed to the next layer. */
void or_mlp_forward(const double *par, const double *x, long nb, int bf16, double *z, double *h1,
                    double *h2);
/* BCE-with-logits loss, mean over the batch, positives weighted by pos_weight;
 * grad (3169 values) receives d loss / d params, back-propagated through the
 * forward values of or_mlp_forward (the rounding treated as identity) */
double or_mlp_loss_grad(const double *par, const double *x, const double *y, long nb,
                        double pos_weight, int bf16, double *grad);
/* Adam update (Kingma & Ba 2015) in place: m, v moments, step t >= 1 */
void or_adam(double *par, const double *grad, double *m, double *v, long n, long t, double lr,
             double b1, double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif
