/*
 * dg.h -- C ABI of the MI355X (gfx950) modal discontinuous Galerkin library.
 *
 * The library advances the 2D compressible Euler equations with stellar and
 * planetary gravity (Velasco Romero et al. 2018, Sec. 2.1 eq. (1)) by the
 * modal DG semi-discretisation of Sec. 2.2 eq. (3) and the SSP Runge-Kutta
 * march of Algorithm 1 (Appendix A, SSP(3,3)).  All compute runs in HIP
 * kernels on the caller's stream; nothing here takes or returns framework
 * (PyTorch) types.
 *
 * Data layout (caller-owned device arrays, FP64):
 *   state  element-tiled: the elements of row j are grouped in tiles of
 *          W = 64 / n consecutive elements (n = order): tile t = j * TX + i / W
 *          with TX = ceil(nx / W), slot s = i % W; inside a tile the entries
 *          run [v][b][a][s], so mode (a, b) of variable v (rho, rho vx,
 *          rho vy[, E]) of element (i, j) is
 *              u[((t * nvar + v) * n + b) * n * W + a * W + s].
 *          Slots past the end of a row are padding: dg_init zeroes them in
 *          u0_dev, and no call reads them or writes them in an output (an
 *          output array keeps whatever its padding held).  The array holds
 *          dg_state_size(cfg) doubles.  (The paper keeps one matrix per mode,
 *          Sec. 3.1; tiles keep what one wavefront reads contiguous.)
 *   basis  phi_ab(xi, eta) = sqrt((2a+1)(2b+1)) P_a(xi) P_b(eta), orthonormal
 *          under (1/|K|) int_K, so mode 00 is the element mean (Sec. 2.2 and
 *          the zeroth-mode statement of Sec. 3.1).
 *   nodes  Gauss-Legendre points, n per direction: node (q, r), flat q*n + r.
 *
 * Errors: every call returns 0 or a negative DG_E* code and never aborts or
 * throws; dg_last_error() gives the message of the last failure of a handle
 * (or of dg_init / dg_get_nodes when the handle is NULL).  Device-side
 * problems (non-finite or non-positive density means) raise a flag that the
 * next dg_sync() reports as DG_ENONFINITE.  A handle belongs to one stream and
 * is not thread-safe.  Process-wide state: the message of the last failed
 * handle-less call, kept per host thread, and the static device array of
 * dg_torque_noalloc (one per GPU) with its device addresses.
 */
#ifndef DG_MI355X_H
#define DG_MI355X_H

#ifdef __cplusplus
extern "C" {
#endif

#define DG_OK 0
#define DG_EINVAL -1        /* bad argument or configuration */
#define DG_ENOMEM -2        /* device allocation failed */
#define DG_EHIP -3          /* a HIP runtime call failed */
#define DG_EUNSUPPORTED -4  /* valid but not built (e.g. order outside 2..5) */
#define DG_ENONFINITE -5    /* device flagged a non-finite / non-positive mean */

enum { DG_CLOSURE_ISOTHERMAL = 0, DG_CLOSURE_LOCALLY_ISOTHERMAL = 1, DG_CLOSURE_ADIABATIC = 2 };
/* box edges: periodic; fixed (exterior trace = the element's initial trace,
 * Sec. 3.1 ghost cells for the disc); gradient-free (Sec. 4.2: a ghost element
 * without gradient, i.e. the exterior state is the element's own current
 * mean) */
enum { DG_BC_PERIODIC = 0, DG_BC_FIXED_INITIAL = 1, DG_BC_GRADIENT_FREE = 2 };
enum { DG_PRECISION_FP64 = 0, DG_PRECISION_MIXED = 1 };
enum { DG_LIMITER_NONE = 0, DG_LIMITER_MODAL_DECAY = 1, DG_LIMITER_LEARNED = 2 };
/* Runge-Kutta tables of Appendix A: SSP(3,3) with c_3 = 1/2 (the default),
 * SSP(2,2) as Heun (a_21 = c_2 = 1), the five-stage fourth-order SSP table
 * and the six-stage Cash-Karp table with its fifth-order weights, both as
 * printed. */
enum { DG_RK_SSP33 = 0, DG_RK_SSP22 = 1, DG_RK_SSP54 = 2, DG_RK_CASHKARP = 3 };
/* Numerical flux of eq. (3) (its type is not named in the paper): Rusanov
 * (local Lax-Friedrichs, the default) or, for the adiabatic closure, HLLC
 * (Toro, Spruce & Speares 1994, with the wave-speed estimates of Davis 1988),
 * which keeps contact and shear waves. */
enum { DG_FLUX_RUSANOV = 0, DG_FLUX_HLLC = 1 };

/* Problem statement.  Units: G = M_* = r_p = 1 as in Sec. 5.1. */
typedef struct dg_config {
    int order;            /* n = N_p + 1 points/modes per direction, 2..5 */
    int nvar;             /* 3 (isothermal closures) or 4 (adiabatic) */
    int nx, ny;           /* elements per direction */
    double x0, x1, y0, y1;/* box */
    int closure;          /* DG_CLOSURE_* */
    double cs;            /* isothermal sound speed */
    double h;             /* aspect ratio: c_s^2 = h^2 GM / max(r, r_core) */
    double gamma;         /* adiabatic index */
    int bc;               /* DG_BC_* */
    int star;             /* 1: stellar potential, harmonic core inside r_core */
    double gm, r_core;
    double q, eps;        /* planet mass ratio (0: no planet) and softening */
    double rp, phi0;      /* planet orbit radius, phase at t = 0 */
    int damping;          /* 1: wave-killing zones r < rd_in and r > rd_out */
    double rd_in, rd_out;
    double cfl;           /* C of the CFL condition (Sec. 2.3) */
    int precision;        /* DG_PRECISION_* */
    double sigma0;        /* deviation form: equilibrium disc Sigma0 (see dg_init) */
    int limiter;          /* DG_LIMITER_* */
    double limiter_s0;    /* modal-decay threshold on log10 of the top-mode energy share */
    double mlp_theta;     /* learned indicator: flag when sigmoid output > theta */
    int rk;               /* DG_RK_* (0 = SSP(3,3)) */
    int positivity;       /* 1: positivity-preserving limiter (Sec. 2.4), see dg_positivity */
    double pp_eps;        /* floor e0 of its eps (<= 0: 1e-13, Zhang & Shu's value) */
    int flux;             /* DG_FLUX_* (DG_FLUX_HLLC: adiabatic closure, FP64 form) */
} dg_config;

typedef struct dg_handle dg_handle;

/* Number of doubles in one state array of this configuration (padding
 * included), or a negative DG_E* code for an invalid configuration.  A state
 * array may hold at most 2^31 - 1 bytes (the kernels address it through
 * buffer resources of that range): larger configurations give
 * DG_EUNSUPPORTED here and in dg_init.  Needs no device. */
long long dg_state_size(const dg_config *cfg);

/* Volume Gauss node coordinates, host arrays x_host[e*n*n + node] and y_host
 * likewise (E*n*n doubles each, caller-owned).  Needs no device. */
int dg_get_nodes(const dg_config *cfg, double *x_host, double *y_host);

/* Initial conditions (Sec. 3.1 steps (i)(a)-(c)).  prim_nodes_host holds the
 * primitive variables (rho, vx, vy[, p]) at the volume nodes, layout
 * [var][e][node], host memory read during the call only.  The projected modes
 * are written to the caller's device array u0_dev (layout above) on
 * hip_stream (a hipStream_t; NULL = default stream), and the library keeps its
 * own copy as the fixed exterior state and the damping target.  The handle
 * owns all workspace it allocates; dg_free releases it.
 *
 * Deviation form (precision DG_PRECISION_MIXED; locally isothermal disc with
 * stellar gravity only): the state is written as u = u_eq + du about the
 * rotational equilibrium of the disc set-up (Sec. 5.1 with the readings of
 * the Sigma profile and harmonic core: Sigma = sigma0 max(r, r_core)^(-1/2),
 * v_phi^2 = r dPhi_star/dr + (r/Sigma) d(c_s^2 Sigma)/dr), projected in FP64 by the
 * library.  Every state array of the handle (u0_dev, the u_dev of dg_rhs,
 * dg_rk_step, dg_torque) then holds the FP64 deviation du, and dg_rhs returns
 * L(u_eq + du); dg_full_state reconstructs u.  The right-hand side is
 * L(u_eq) (FP64, computed once and kept) plus the deviation part
 * L(u_eq + du) - L(u_eq) in FP32, every deviation flux linearised about u_eq's
 * own polynomial (its values at the volume nodes and its edge traces, the
 * latter tabulated in FP32 at init). */
int dg_init(const dg_config *cfg, const double *prim_nodes_host, double *u0_dev, void *hip_stream,
            dg_handle **out);

/* Deviation form only: full = u_eq + dev (device arrays, state layout; they
 * may alias).  FP64 mode: full = dev. */
int dg_full_state(dg_handle *h, const double *dev_dev, double *full_dev);

/* Right-hand side of eq. (3), rhs = L(u) at time t (planet at its position
 * at t), without limiter or damping.  u_dev, rhs_dev: device arrays in the
 * state layout, distinct.  Asynchronous on the handle's stream. */
int dg_rhs(dg_handle *h, double t, const double *u_dev, double *rhs_dev);

/* One Runge-Kutta step (Algorithm 1) of the state u_dev, in place, with the
 * table cfg->rk (default SSP(3,3), c = (0, 1, 1/2), run in Shu-Osher form;
 * the other tables in Butcher form: stage derivatives k_i = L(y_i, t^n + c_i
 * dt) kept in handle-owned buffers, y_i = u^n + dt sum_j a_ij k_j).  t_dev is
 * a device double holding t^n; it is advanced to t^n + dt on the device.
 * dt = dt_fixed if dt_fixed > 0, else the CFL step of Sec. 2.3 from the
 * element means of u^n, reduced on the device.  dt_used_dev (device double,
 * may be NULL) receives dt.  The limiter (if configured; SSP(3,3) only, else
 * dg_init returns DG_EUNSUPPORTED) is applied to every stage state after its
 * update, the damping once after the last stage.  No host synchronisation. */
int dg_rk_step(dg_handle *h, double *u_dev, double *t_dev, double dt_fixed, double *dt_used_dev);

/* z-torque of the disc on the planet, eq. (5) (G = 1, per unit planet mass),
 * with the cells read as the volume Gauss nodes (mass rho_h w_q w_r |K| / 4).
 * Time: *t_dev if t_dev is not NULL, else t.  The result is written to the
 * device double torque_dev; the summation order is fixed, so repeated calls
 * give identical bits. */
int dg_torque(dg_handle *h, double t, const double *t_dev, const double *u_dev, double *torque_dev);

/* The torque of eq. (5) of the state entering the step (u^n at t^n, as
 * dg_torque(h, 0, t_dev, u_dev, torque_dev) before the step gives it), then one
 * step of dg_rk_step (Algorithm 1): the same torque bits and the same state.
 * Sec. 5.2 records the torque every step; here the first stage kernel forms it
 * from the node densities and planet offsets it evaluates anyway (one partial
 * per tile), and one more block of the last stage launch adds the partials up
 * in the same fixed order as dg_torque; this saves the torque kernel's read
 * of the density and the launch of the final sum.  The deviation form, and the positivity
 * limiter without a troubled-cell limiter (its scaling fused into the stage
 * kernels), run the two calls one after the other.  After the last step, dg_torque gives the torque of the
 * final state.  torque_dev: device double.  Errors as for dg_rk_step. */
int dg_rk_step_torque(dg_handle *h, double *u_dev, double *t_dev, double dt_fixed, double *dt_used_dev,
                      double *torque_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the torque of
 * dg_torque, same kernels, same bits, without a handle.  cfg describes the
 * state (FP64 form only: DG_PRECISION_MIXED gives DG_EUNSUPPORTED); u_dev,
 * t_dev (may be NULL: then t) and torque_dev are device memory as in
 * dg_torque; the work is queued on hip_stream (NULL = default stream).  The
 * per-tile partial sums live in a static device array of 524288 doubles
 * (4 MiB per GPU, held until the process ends): grids of more than 524288
 * tiles of 64 / order elements of a row give DG_EUNSUPPORTED.
 * Nothing is allocated and no state is kept between calls except that array:
 * calls that overlap on one GPU (other streams, other host threads) race on
 * it, so the caller serialises them.  Errors as for the handle-less calls
 * (dg_last_error(NULL)). */
int dg_torque_noalloc(const dg_config *cfg, double t, const double *t_dev, const double *u_dev, double *torque_dev,
                      void *hip_stream);

/* ---- troubled cells (limiter DG_LIMITER_MODAL_DECAY or DG_LIMITER_LEARNED) ----
 *
 * The limiter is the minmod slope limiter of the Cockburn-Shu RKDG scheme the
 * paper follows (Sec. 2.2): on a troubled element the linear modes are
 * replaced by minmod(own slope, forward and backward differences of the
 * neighbour means), component-wise per conservative variable; if any slope
 * changes, every higher mode is dropped.  Means are never changed.  The plain
 * indicator flags an element when log10 of the share of its density energy
 * in the modes of top degree (max(a, b) = N_p) exceeds cfg->limiter_s0.  The
 * learned indicator is a 64 -> 32 -> 32 -> 1 MLP (ReLU, sigmoid output; bf16
 * weights and inputs, FP32 accumulation on MFMA) on the element features
 * f[v*16 + m] = u_vm / (|u_v00| + s_v) (order 4, four variables); it flags
 * when the sigmoid exceeds cfg->mlp_theta.  With a limiter configured,
 * dg_rk_step limits each stage state after its update (Shu-Osher form). */

/* Plain indicator and minmod on u_dev: apply != 0 limits in place.  Outputs
 * (device arrays of E entries, each may be NULL): flag_dev (indicator fired),
 * changed_dev (minmod alters a slope: the training label), sensor_dev (log10
 * energy share, float). */
int dg_troubled(dg_handle *h, double *u_dev, int apply, unsigned char *flag_dev, unsigned char *changed_dev,
                float *sensor_dev);
/* Positivity-preserving limiter of Sec. 2.4 (the scaling limiter of Zhang &
 * Shu 2010), in place on every element of u_dev (device, the layout above).
 * Test points of an element: the tensor sets (Gauss-Lobatto in x) x (Gauss in
 * y) and (Gauss in x) x (Gauss-Lobatto in y), with the fewest Lobatto points L
 * such that 2L - 3 >= N_p.  eps = min(e0, mean density, mean pressure), e0 =
 * cfg->pp_eps (1e-13 when <= 0).
 * The density's non-mean modes are scaled by theta1 = (mean - eps) / (mean -
 * min) where its minimum over the points is below eps; then (adiabatic closure
 * only) every variable's non-mean modes by theta2, the smallest over the
 * points w whose pressure is below eps of the largest t in [0, 1] with
 * p(mean + t (w - mean)) >= eps (bisection, keeping the admissible end).  Means never change; elements whose means are not admissible are left
 * alone.  Outputs (device, may be NULL): changed_dev[e] (E bytes) = 1 where a
 * mode changed, theta_dev[2e], theta_dev[2e+1] (2E doubles) = theta1, theta2.
 * With cfg->positivity = 1 (SSP(3,3), FP64 form), dg_init limits the projected
 * initial state, dg_rk_step limits every stage state after the minmod limiter
 * (if any) and the damped state after the damping, and the CFL factor C/(2N_p+1) becomes C min(1/(2N_p+1), w_1/2),
 * w_1 the end weight of the Lobatto rule normalised to sum 1. */
int dg_positivity(dg_handle *h, double *u_dev, unsigned char *changed_dev, double *theta_dev);
/* Feature scales s_v (RMS of the initial element means of variable v), host
 * array of nvar doubles. */
int dg_mlp_feature_scales(dg_handle *h, double *scales_host);
/* bf16 features of every element, feat_dev[e*64 + v*16 + m] (needs order 4,
 * nvar 4). */
int dg_mlp_features(dg_handle *h, const double *u_dev, unsigned short *feat_dev);
/* Set (set_host != NULL; resets the Adam moments and step) and/or read
 * (get_host != NULL) the 3169 FP32 master parameters, layout W1[32][64], b1[32],
 * W2[32][32], b2[32], w3[32], b3.  Host arrays. */
int dg_mlp_params(dg_handle *h, const float *set_host, float *get_host);
/* Logits of n feature rows (device arrays). */
int dg_mlp_forward(dg_handle *h, const unsigned short *feat_dev, long n, float *logit_dev);
/* One training step on n samples: forward, BCE-with-logits (mean, positives
 * weighted by pos_weight) backward, and Adam (beta 0.9 / 0.999, eps 1e-8) with
 * learning rate lr (lr <= 0: gradient only, parameters unchanged).  loss_dev
 * (1 float) and grad_dev (3169 floats) may be NULL.  Device arrays; the
 * handle keeps the workspace for the largest n seen. */
int dg_mlp_train_step(dg_handle *h, const unsigned short *feat_dev, const float *label_dev, long n, float pos_weight,
                      float lr, float *loss_dev, float *grad_dev);

/* One-shot capture for training data and indicator evaluation: the next
 * dg_rk_step records, for the state of its last stage before limiting, the bf16
 * features (feat_dev, E x 64), the plain indicator's flags (flag_dev) and
 * labels (label_dev: flagged and minmod alters a slope), and with the learned
 * limiter its flags (mlp_flag_dev).  Device arrays of E entries; any may be
 * NULL.  Needs a configured limiter. */
int dg_capture(dg_handle *h, unsigned short *feat_dev, unsigned char *flag_dev, unsigned char *label_dev,
               unsigned char *mlp_flag_dev);

/* Wait for the handle's stream; returns DG_ENONFINITE if a kernel flagged a
 * non-finite or non-positive density mean since the last dg_sync. */
int dg_sync(dg_handle *h);

/* Kernel timing for measurement: between dg_profile_begin and dg_profile_end
 * every launch of the fused RK-stage kernel issued by dg_rk_step is bracketed
 * by HIP events on the handle's stream.  dg_profile_end waits for them and
 * returns the summed duration (ms) and the number of launches. */
int dg_profile_begin(dg_handle *h);
int dg_profile_end(dg_handle *h, double *stage_ms, int *stage_launches);

/* Release the handle and its workspace (NULL is accepted). */
int dg_free(dg_handle *h);

/* Message of the last error of h (NULL: of the last failed handle-less call). */
const char *dg_last_error(const dg_handle *h);

#ifdef __cplusplus
}
#endif
#endif
