// C ABI of the gfx950 DG library (declarations and contracts in include/dg.h).
#include "../../include/dg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dg_basis.h"
#include "dg_internal.h"

using dgk::Geo;
using dgk::StageCoeffs;
using dgk::StepBlock;

struct dg_handle {
    dg_config cfg{};
    int n = 0, nvar = 0;
    long long E = 0;
    Geo g{};
    hipStream_t s = nullptr;
    int device = 0;
    double* u0 = nullptr;   // initial modes (full state): fixed exterior state and damping target
    bool dev = false;       // deviation form (DG_PRECISION_MIXED)
    double* eq = nullptr;   // deviation form: projected equilibrium u_eq (FP64)
    double* du0 = nullptr;  // deviation form: initial deviation (fixed exterior state)
    double* leq = nullptr;  // deviation form: L(u_eq) without the planet (FP64)
    float* eqtr = nullptr;  // deviation form: u_eq's traces at the edge points (FP32)
    double* ws1 = nullptr;  // SSP stage states u^(1), u^(2); Butcher stage state y_i
    double* ws2 = nullptr;
    dgk::RKTable tab{};     // Butcher tables (DG_RK_SSP54, DG_RK_CASHKARP)
    double* kbuf = nullptr; // their stage derivatives k_1 .. k_s
    StageCoeffs* sc_rhs = nullptr;
    StepBlock* sb = nullptr;
    double* dt_part = nullptr;        // per-block CFL minima
    unsigned int* bad_part = nullptr; // per-block flags
    int dt_blocks = 0;
    int* damp_list = nullptr;
    int ndamp = 0;
    double* damp_q0 = nullptr;  // damping targets at the Gauss nodes of the listed tiles
    double* tq_part = nullptr;  // torque partials, one per tile
    bool rev = false;           // tile direction of the next stage launch (alternates)
    // troubled cells / learned indicator
    double* scale_dev = nullptr;     // feature scales (nvar)
    double scale_host[4] = {0, 0, 0, 0};
    unsigned char* flags = nullptr;  // E
    unsigned short* feat = nullptr;  // E * 64 (learned limiter)
    float* mlp = nullptr;            // parameters, Adam m, Adam v (3 * nparam)
    void* mlp_pack = nullptr;        // the weights in per-lane fragment form (learned limiter)
    unsigned char* pp_ok = nullptr;  // per tile: no positivity scaling needed (limiter + positivity, order 4 adiabatic)
    unsigned char* undamped = nullptr;  // per tile: not touched by the damping (positivity + damping)
    long long adam_t = 0;
    long long tr_cap = 0;            // training workspace capacity (samples)
    float* tr_ws = nullptr;          // z, h1, h2, dz, d1, d2, loss partials, grad
    bool cap = false;                // one-shot capture armed for the next step's last stage
    unsigned short* cap_feat = nullptr;
    unsigned char *cap_flag = nullptr, *cap_label = nullptr, *cap_mlp = nullptr;
    bool prof = false;               // bracket stage launches with events
    std::vector<hipEvent_t> ev;      // start/stop pairs
    std::string err;
};

namespace {

thread_local std::string g_err;  // last error of a handle-less call

int fail(dg_handle* h, int code, const std::string& msg) {
    if (h)
        h->err = msg;
    else
        g_err = msg;
    return code;
}

int hip_fail(dg_handle* h, hipError_t e, const char* what) {
    return fail(h, DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define DG_HIP(h, call, what)                                  \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail((h), e_, (what)); \
    } while (0)

// elements of the tiled layout, padding included
double state_slots(const dg_config* c) {
    const int ew = dgk::tile_width(c->order);
    return (double)((c->nx + ew - 1) / ew) * ew * (double)c->ny;
}

int validate(const dg_config* c, std::string* why) {
    if (!c) return (*why = "cfg is NULL", DG_EINVAL);
    if (c->order < 2 || c->order > dgk::kMaxN) return (*why = "order must be in 2..5", DG_EUNSUPPORTED);
    if (c->nx < 1 || c->ny < 1) return (*why = "nx, ny must be >= 1", DG_EINVAL);
    if ((long long)c->nx * c->ny > (1LL << 31) - 1) return (*why = "too many elements", DG_EINVAL);
    if (!(c->x1 > c->x0) || !(c->y1 > c->y0)) return (*why = "empty box", DG_EINVAL);
    if (c->closure < 0 || c->closure > 2) return (*why = "unknown closure", DG_EINVAL);
    if (c->nvar != (c->closure == DG_CLOSURE_ADIABATIC ? 4 : 3))
        return (*why = "nvar must be 4 for the adiabatic closure and 3 otherwise", DG_EINVAL);
    if (c->closure == DG_CLOSURE_ISOTHERMAL && !(c->cs > 0)) return (*why = "cs must be > 0", DG_EINVAL);
    if (c->closure == DG_CLOSURE_LOCALLY_ISOTHERMAL && !(c->h > 0 && c->gm > 0 && c->r_core > 0))
        return (*why = "h, gm, r_core must be > 0", DG_EINVAL);
    if (c->closure == DG_CLOSURE_ADIABATIC && !(c->gamma > 1)) return (*why = "gamma must be > 1", DG_EINVAL);
    if (c->bc != DG_BC_PERIODIC && c->bc != DG_BC_FIXED_INITIAL && c->bc != DG_BC_GRADIENT_FREE)
        return (*why = "unknown bc", DG_EINVAL);
    if (c->bc == DG_BC_GRADIENT_FREE && c->precision != DG_PRECISION_FP64)
        return (*why = "the gradient-free box edge is built for the FP64 form", DG_EUNSUPPORTED);
    if (c->star && !(c->gm > 0 && c->r_core > 0)) return (*why = "star needs gm, r_core > 0", DG_EINVAL);
    if (c->q < 0 || (c->q > 0 && !(c->eps > 0 && c->rp > 0 && c->gm > 0)))
        return (*why = "planet needs q >= 0, eps, rp, gm > 0", DG_EINVAL);
    if (c->damping && !(c->rd_in >= 0 && c->rd_out > c->rd_in && c->gm > 0))
        return (*why = "damping needs 0 <= rd_in < rd_out and gm > 0", DG_EINVAL);
    if (!(c->cfl > 0)) return (*why = "cfl must be > 0", DG_EINVAL);
    if (c->precision != DG_PRECISION_FP64 && c->precision != DG_PRECISION_MIXED)
        return (*why = "unknown precision", DG_EINVAL);
    if (c->precision == DG_PRECISION_MIXED &&
        !(c->closure == DG_CLOSURE_LOCALLY_ISOTHERMAL && c->star && c->sigma0 > 0))
        return (*why = "the deviation form is built for the locally isothermal disc with stellar gravity and sigma0 > 0",
                DG_EUNSUPPORTED);
    if (c->limiter < DG_LIMITER_NONE || c->limiter > DG_LIMITER_LEARNED) return (*why = "unknown limiter", DG_EINVAL);
    if (c->rk < DG_RK_SSP33 || c->rk > DG_RK_CASHKARP) return (*why = "unknown Runge-Kutta table", DG_EINVAL);
    if (c->rk != DG_RK_SSP33 && c->limiter != DG_LIMITER_NONE)
        return (*why = "limiters are built for the SSP(3,3) table", DG_EUNSUPPORTED);
    if (c->limiter != DG_LIMITER_NONE && c->precision != DG_PRECISION_FP64)
        return (*why = "limiters are built for the FP64 form", DG_EUNSUPPORTED);
    if (c->limiter == DG_LIMITER_LEARNED && !(c->order == 4 && c->nvar == 4))
        return (*why = "the learned indicator takes 16 modes x 4 variables (order 4, nvar 4)", DG_EUNSUPPORTED);
    if (c->limiter == DG_LIMITER_LEARNED && !(c->mlp_theta > 0 && c->mlp_theta < 1))
        return (*why = "mlp_theta must be in (0, 1)", DG_EINVAL);
    if (c->positivity != 0 && c->positivity != 1) return (*why = "positivity must be 0 or 1", DG_EINVAL);
    if (!(c->pp_eps >= 0 && c->pp_eps < 1e300)) return (*why = "pp_eps must be finite and >= 0", DG_EINVAL);
    if (c->positivity && c->rk != DG_RK_SSP33)
        return (*why = "the positivity limiter is built for the SSP(3,3) table", DG_EUNSUPPORTED);
    if (c->positivity && c->precision != DG_PRECISION_FP64)
        return (*why = "the positivity limiter is built for the FP64 form", DG_EUNSUPPORTED);
    if (c->flux != DG_FLUX_RUSANOV && c->flux != DG_FLUX_HLLC) return (*why = "unknown flux", DG_EINVAL);
    if (c->flux == DG_FLUX_HLLC && !(c->closure == DG_CLOSURE_ADIABATIC && c->precision == DG_PRECISION_FP64))
        return (*why = "the HLLC flux is built for the adiabatic closure in the FP64 form", DG_EUNSUPPORTED);
    // the kernels address state arrays through buffer resources whose range
    // is 2^31 - 1 bytes
    if ((double)c->nvar * c->order * c->order * state_slots(c) * 8.0 > 2147483647.0)
        return (*why = "state arrays are limited to 2^31 - 1 bytes (buffer-resource range)", DG_EUNSUPPORTED);
    return DG_OK;
}

void make_geo(const dg_config* c, Geo* g) {
    *g = Geo{};
    g->nx = c->nx;
    g->ny = c->ny;
    g->E = (long long)c->nx * c->ny;
    g->ew = dgk::tile_width(c->order);
    g->tiles_x = (c->nx + g->ew - 1) / g->ew;
    g->slots = (long long)g->tiles_x * c->ny * g->ew;
    g->x0 = c->x0;
    g->y0 = c->y0;
    g->dx = (c->x1 - c->x0) / c->nx;
    g->dy = (c->y1 - c->y0) / c->ny;
    g->rdx2 = 2.0 / g->dx;
    g->rdy2 = 2.0 / g->dy;
    g->idx = 1.0 / g->dx;
    g->idy = 1.0 / g->dy;
    g->closure = c->closure;
    g->bc = c->bc;
    g->star = c->star;
    g->cs2 = c->cs * c->cs;
    g->cs = c->cs;
    g->rc2 = c->r_core * c->r_core;
    g->irc = c->r_core > 0 ? 1.0 / c->r_core : 0.0;
    g->h2gm = c->h * c->h * c->gm;
    g->gamma = c->gamma;
    g->gm = c->gm;
    g->r_core = c->r_core;
    g->rc3inv = c->r_core > 0 ? c->gm / (c->r_core * c->r_core * c->r_core) : 0.0;
    g->q = c->q;
    g->eps2 = c->eps * c->eps;
    g->gm_h = g->gm * (0.5 * g->dx);
    g->rc3inv_h = g->rc3inv * (0.5 * g->dx);
    g->q_h = g->q * (0.5 * g->dx);
    g->rp = c->rp;
    g->phi0 = c->phi0;
    g->omp = c->rp > 0 ? std::sqrt(c->gm / (c->rp * c->rp * c->rp)) : 0.0;
    g->damping = c->damping;
    const double f = std::pow(1.15, 1.5);
    const double pi = 3.141592653589793238462643;
    g->rd_in = c->rd_in;
    g->rd_out = c->rd_out;
    g->rb_in = c->rd_in / f;
    g->rb_out = c->rd_out * f;
    g->irw_in = 1.0 / (g->rb_in - g->rd_in);
    g->irw_out = 1.0 / (g->rb_out - g->rd_out);
    g->td_in = c->gm > 0 ? 2.0 * pi * std::sqrt(c->rd_in * c->rd_in * c->rd_in / c->gm) : 0.0;
    g->td_out = c->gm > 0 ? 2.0 * pi * std::sqrt(c->rd_out * c->rd_out * c->rd_out / c->gm) : 0.0;
    g->cfl_fac = c->cfl / (2.0 * (c->order - 1) + 1.0);
    g->pp_eps = c->pp_eps > 0.0 ? c->pp_eps : 1e-13;
    g->flux = c->flux;
    if (c->positivity) {
        // Sec. 2.4: C min(1/(2N_p+1), w_1/2), w_1 of the limiter's Lobatto rule
        const dgk::LobattoTab lt = dgk::make_lobatto(c->order);
        g->cfl_fac = c->cfl * std::fmin(1.0 / (2.0 * (c->order - 1) + 1.0), lt.w1h);
    }
    g->sigma0 = c->sigma0;
}


void host_nodes(const dg_config* c, std::vector<double>* x, std::vector<double>* y) {
    const int n = c->order;
    const dgk::BasisTab T = dgk::make_basis(n);
    const double dx = (c->x1 - c->x0) / c->nx, dy = (c->y1 - c->y0) / c->ny;
    const long long E = (long long)c->nx * c->ny;
    x->resize((size_t)E * n * n);
    y->resize((size_t)E * n * n);
    for (long long e = 0; e < E; ++e) {
        const int i = (int)(e % c->nx), j = (int)(e / c->nx);
        const double xc = c->x0 + (i + 0.5) * dx, yc = c->y0 + (j + 0.5) * dy;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r) {
                (*x)[(size_t)e * n * n + q * n + r] = xc + 0.5 * dx * T.xi[q];
                (*y)[(size_t)e * n * n + q * n + r] = yc + 0.5 * dy * T.xi[r];
            }
    }
}

void drop_events(dg_handle* h) {
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    h->ev.clear();
}

// launch one stage kernel, bracketed by events while profiling; pp: with the
// positivity scaling fused (FP64 path)
hipError_t stage(dg_handle* h, const double* u, const double* un, double* out, const StageCoeffs* sc,
                 bool pp = false, double* tq_part = nullptr, const dgk::MlpFlags* mf = nullptr,
                 unsigned char* pp_ok = nullptr, double* tq_out = nullptr) {
    hipEvent_t a = nullptr, b = nullptr;
    if (h->prof) {
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
        h->ev.push_back(a);
        h->ev.push_back(b);
        e = hipEventRecord(a, h->s);
        if (e != hipSuccess) return e;
    }
    // each launch walks the tiles in the direction opposite to the last one
    const bool rev = h->rev;
    h->rev = !h->rev;
    hipError_t e = h->dev ? dgk::launch_stage_dev(h->n, h->g, u, un, h->du0, h->leq, h->eqtr, out, sc, h->s, rev)
                          : dgk::launch_stage(h->n, h->g, u, un, h->u0, out, sc, pp, tq_part, h->s, mf, pp_ok, rev,
                                              tq_out ? h->tq_part : nullptr, tq_out);
    if (e == hipSuccess && h->prof) e = hipEventRecord(b, h->s);
    return e;
}

// primitive node values of the disc's rotational equilibrium (reading of the
// Sec. 5.1 set-up: Sigma = sigma0 max(r, r_core)^(-1/2), locally isothermal
// pressure, harmonic stellar core), layout [var][e][node]
void equilibrium_prim(const dg_config* c, std::vector<double>* prim) {
    std::vector<double> x, y;
    host_nodes(c, &x, &y);
    const size_t M = x.size();
    prim->assign(3 * M, 0.0);
    for (size_t k = 0; k < M; ++k) {
        const double r = std::sqrt(x[k] * x[k] + y[k] * y[k]);
        const double rr = r > c->r_core ? r : c->r_core;
        const double om2 = r < c->r_core ? c->gm / (c->r_core * c->r_core * c->r_core)
                                         : c->gm * (1.0 - 1.5 * c->h * c->h) / (r * r * r);
        const double om = std::sqrt(om2);
        (*prim)[k] = c->sigma0 / std::sqrt(rr);
        (*prim)[M + k] = -om * y[k];
        (*prim)[2 * M + k] = om * x[k];
    }
}

// configured limiter on a stage state, in place; `last` marks the last stage
// of a step (where an armed capture records the pre-limiter state)
hipError_t limit(dg_handle* h, double* u, bool last) {
    const int lim = h->cfg.limiter;
    const int pp = h->cfg.positivity;
    if (lim == DG_LIMITER_NONE)
        return pp ? dgk::launch_troubled(h->n, h->nvar, h->g, u, h->u0, 0.0, 2, 1, nullptr, nullptr, nullptr, nullptr,
                                         1, nullptr, h->s)
                  : hipSuccess;
    hipError_t e = hipSuccess;
    const bool cap = last && h->cap;
    if (cap) {
        h->cap = false;
        if (h->cap_feat) e = dgk::launch_features(h->n, h->nvar, h->g, u, h->scale_dev, h->cap_feat, h->s);
        if (e == hipSuccess && (h->cap_flag || h->cap_label))
            e = dgk::launch_troubled(h->n, h->nvar, h->g, u, h->u0, h->cfg.limiter_s0, 0, 0, nullptr, h->cap_flag,
                                     h->cap_label, nullptr, 0, nullptr, h->s);
        if (e != hipSuccess) return e;
    }
    if (lim == DG_LIMITER_MODAL_DECAY)
        return dgk::launch_troubled(h->n, h->nvar, h->g, u, h->u0, h->cfg.limiter_s0, 0, 1, nullptr, nullptr, nullptr,
                                    nullptr, pp, nullptr, h->s, h->pp_ok);
    // the learned indicator's flags of u were formed by the stage kernel that
    // wrote u
    if (e == hipSuccess && cap && h->cap_mlp)
        e = hipMemcpyAsync(h->cap_mlp, h->flags, (size_t)h->E, hipMemcpyDeviceToDevice, h->s);
    if (e == hipSuccess)
        e = dgk::launch_troubled(h->n, h->nvar, h->g, u, h->u0, 0.0, 1, 1, h->flags, nullptr, nullptr, nullptr, pp,
                                 nullptr, h->s, h->pp_ok);
    return e;
}

// Butcher tables of Appendix A run in Butcher form: the five-stage
// fourth-order SSP table and Cash-Karp (fifth-order weights), as printed
void butcher_table(int rk, dgk::RKTable* t) {
    *t = dgk::RKTable{};
    constexpr int M = dgk::kMaxStages;
    if (rk == DG_RK_SSP54) {
        const double a[5][4] = {{0, 0, 0, 0},
                                {0.39175222700392, 0, 0, 0},
                                {0.21766909633821, 0.36841059262959, 0, 0},
                                {0.08269208670950, 0.13995850206999, 0.25189177424738, 0},
                                {0.06796628370320, 0.11503469844438, 0.20703489864929, 0.54497475021237}};
        const double b[5] = {0.14681187618661, 0.24848290924556, 0.10425883036650, 0.27443890091960,
                             0.22600748319395};
        const double c[5] = {0, 0.39175222700392, 0.58607968896779, 0.47454236302687, 0.93501063100924};
        t->s = 5;
        for (int i = 0; i < 5; ++i) {
            for (int j = 0; j < 4; ++j) t->A[i * M + j] = a[i][j];
            t->b[i] = b[i];
            t->c[i] = c[i];
        }
    } else if (rk == DG_RK_CASHKARP) {
        const double a[6][5] = {{0, 0, 0, 0, 0},
                                {1.0 / 5, 0, 0, 0, 0},
                                {3.0 / 40, 9.0 / 40, 0, 0, 0},
                                {3.0 / 10, -9.0 / 10, 6.0 / 5, 0, 0},
                                {-11.0 / 54, 5.0 / 2, -70.0 / 27, 35.0 / 27, 0},
                                {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592, 253.0 / 4096}};
        const double b[6] = {37.0 / 378, 0, 250.0 / 621, 125.0 / 594, 0, 512.0 / 1771};
        const double c[6] = {0, 1.0 / 5, 3.0 / 10, 3.0 / 5, 1, 7.0 / 8};
        t->s = 6;
        for (int i = 0; i < 6; ++i) {
            for (int j = 0; j < 5; ++j) t->A[i * M + j] = a[i][j];
            t->b[i] = b[i];
            t->c[i] = c[i];
        }
    }
}

void release(dg_handle* h) {
    if (!h) return;
    drop_events(h);
    (void)hipFree(h->u0);
    (void)hipFree(h->ws1);
    (void)hipFree(h->ws2);
    (void)hipFree(h->sc_rhs);
    (void)hipFree(h->sb);
    (void)hipFree(h->dt_part);
    (void)hipFree(h->bad_part);
    h->dt_part = nullptr;
    h->bad_part = nullptr;
    (void)hipFree(h->damp_list);
    (void)hipFree(h->damp_q0);
    (void)hipFree(h->tq_part);
    h->tq_part = nullptr;
    (void)hipFree(h->eq);
    (void)hipFree(h->du0);
    (void)hipFree(h->leq);
    (void)hipFree(h->eqtr);
    (void)hipFree(h->scale_dev);
    (void)hipFree(h->flags);
    (void)hipFree(h->feat);
    (void)hipFree(h->mlp);
    (void)hipFree(h->mlp_pack);
    h->mlp_pack = nullptr;
    (void)hipFree(h->pp_ok);
    h->pp_ok = nullptr;
    (void)hipFree(h->undamped);
    h->undamped = nullptr;
    (void)hipFree(h->tr_ws);
    (void)hipFree(h->kbuf);
    h->kbuf = nullptr;
    h->u0 = h->ws1 = h->ws2 = h->eq = h->du0 = nullptr;
    h->leq = nullptr;
    h->eqtr = nullptr;
}

// Scratch of dg_torque_noalloc: the torque's per-tile partial sums (4 MiB),
// one copy per GPU in a static device array (no allocation at any call).
// Host code uses the device address from hipGetSymbolAddress, never the
// array's name (a host-side stand-in).
constexpr int kNoAllocPartials = 1 << 19;
__device__ __align__(256) double scratch[kNoAllocPartials];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// the current device's scratch address, looked up once per device
hipError_t scratch_of_current_device(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int dg_get_nodes(const dg_config* cfg, double* x_host, double* y_host) {
    std::string why;
    if (!cfg || !x_host || !y_host) return fail(nullptr, DG_EINVAL, "NULL argument");
    if (cfg->order < 2 || cfg->order > dgk::kMaxN) return fail(nullptr, DG_EUNSUPPORTED, "order must be in 2..5");
    if (cfg->nx < 1 || cfg->ny < 1) return fail(nullptr, DG_EINVAL, "nx, ny must be >= 1");
    std::vector<double> x, y;
    host_nodes(cfg, &x, &y);
    std::memcpy(x_host, x.data(), x.size() * sizeof(double));
    std::memcpy(y_host, y.data(), y.size() * sizeof(double));
    return DG_OK;
}

long long dg_state_size(const dg_config* cfg) {
    std::string why;
    const int rc = validate(cfg, &why);
    if (rc != DG_OK) {
        g_err = why;
        return rc;
    }
    return (long long)cfg->nvar * cfg->order * cfg->order * (long long)state_slots(cfg);
}

int dg_init(const dg_config* cfg, const double* prim_nodes_host, double* u0_dev, void* hip_stream, dg_handle** out) {
    if (!out) return fail(nullptr, DG_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    int rc = validate(cfg, &why);
    if (rc != DG_OK) return fail(nullptr, rc, why);
    if (!prim_nodes_host || !u0_dev) return fail(nullptr, DG_EINVAL, "NULL prim_nodes_host or u0_dev");

    dg_handle* h = new (std::nothrow) dg_handle();
    if (!h) return fail(nullptr, DG_ENOMEM, "host allocation failed");
    h->cfg = *cfg;
    h->n = cfg->order;
    h->nvar = cfg->nvar;
    h->E = (long long)cfg->nx * cfg->ny;
    h->s = (hipStream_t)hip_stream;
    h->dev = cfg->precision == DG_PRECISION_MIXED;
    make_geo(cfg, &h->g);

    auto bail = [&](int code) {
        g_err = h->err;
        release(h);
        delete h;
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) return bail(hip_fail(h, hipGetLastError(), "hipGetDevice"));

    const size_t state_bytes = sizeof(double) * (size_t)h->nvar * h->n * h->n * (size_t)h->g.slots;
    const size_t prim_bytes = sizeof(double) * (size_t)h->nvar * h->n * h->n * (size_t)h->E;  // [var][e][node]
    double* prim_dev = nullptr;
    hipError_t e;
#define DG_ALLOC(ptr, bytes)                                                   \
    e = hipMalloc((void**)&(ptr), (bytes));                                    \
    if (e != hipSuccess) {                                                     \
        (void)hipFree(prim_dev);                                                     \
        return bail(fail(h, DG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e))); \
    }
    DG_ALLOC(h->u0, state_bytes);
    DG_ALLOC(h->ws1, state_bytes);
    DG_ALLOC(h->ws2, state_bytes);
    DG_ALLOC(h->sc_rhs, sizeof(StageCoeffs));
    DG_ALLOC(h->sb, sizeof(StepBlock));
    h->dt_blocks = dgk::dt_blocks(h->g);
    DG_ALLOC(h->dt_part, sizeof(double) * (size_t)h->dt_blocks);
    DG_ALLOC(h->bad_part, sizeof(unsigned int) * (size_t)h->dt_blocks);
    DG_ALLOC(h->tq_part, sizeof(double) * (size_t)dgk::torque_partials(h->g));
    DG_ALLOC(prim_dev, prim_bytes);
    DG_ALLOC(h->scale_dev, sizeof(double) * 4);
    DG_ALLOC(h->flags, (size_t)h->E);
    DG_ALLOC(h->mlp, sizeof(float) * 3 * (size_t)dgk::mlp_nparam());
    if (cfg->limiter == DG_LIMITER_LEARNED) DG_ALLOC(h->mlp_pack, (size_t)dgk::mlp_pack_bytes());
    if (cfg->limiter != DG_LIMITER_NONE && cfg->positivity && h->n == 4 && cfg->closure == DG_CLOSURE_ADIABATIC)
        DG_ALLOC(h->pp_ok, (size_t)dgk::torque_partials(h->g));  // one byte per tile
    butcher_table(cfg->rk, &h->tab);
    if (h->tab.s > 0) DG_ALLOC(h->kbuf, state_bytes * (size_t)h->tab.s);
    if (h->dev) {
        DG_ALLOC(h->eq, state_bytes);
        DG_ALLOC(h->du0, state_bytes);
        DG_ALLOC(h->leq, state_bytes);
        DG_ALLOC(h->eqtr, sizeof(float) * (size_t)dgk::eq_trace_entries(h->n, h->g));
    }

    // damped tiles: tiles with any volume node of non-zero ramp (the kernel
    // leaves the undamped elements of such a tile unchanged: zero increments)
    if (cfg->damping) {
        std::vector<double> x, y;
        host_nodes(cfg, &x, &y);
        std::vector<int> list;
        const int nn = h->n * h->n;
        const int ew = h->g.ew;
        for (int j = 0; j < cfg->ny; ++j)
            for (int t = 0; t < h->g.tiles_x; ++t) {
                bool any = false;  // the ramp is positive exactly for r < rd_in or r > rd_out
                for (int i = t * ew; i < (t + 1) * ew && i < cfg->nx && !any; ++i) {
                    const long long el = (long long)j * cfg->nx + i;
                    for (int k = 0; k < nn && !any; ++k) {
                        const double r = std::sqrt(x[el * nn + k] * x[el * nn + k] + y[el * nn + k] * y[el * nn + k]);
                        any = r < cfg->rd_in || r > cfg->rd_out;
                    }
                }
                if (any) list.push_back(j * h->g.tiles_x + t);
            }
        // ordered by the tile's place in its XCD band (the stage kernels give
        // XCD x the x-th eighth of the tiles): the damping then follows the
        // last stage's order, or runs against it (it starts where that stage
        // ended, on the tiles it wrote last)
        {
            const long long tot = (long long)h->g.tiles_x * cfg->ny;
            const long long per = tot % 8 == 0 ? tot / 8 : tot;
            std::stable_sort(list.begin(), list.end(), [per](int a, int b) { return a % per < b % per; });
        }
        h->ndamp = (int)list.size();
        if (cfg->positivity) {
            // the positivity pass after the damping looks at the damped tiles
            // only: every other tile left the last stage admissible and the
            // damping did not touch it
            std::vector<unsigned char> und((size_t)dgk::torque_partials(h->g), 1);
            for (int tl : list) und[tl] = 0;
            DG_ALLOC(h->undamped, und.size());
            e = hipMemcpy(h->undamped, und.data(), und.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(prim_dev);
                return bail(hip_fail(h, e, "undamped tile marks upload"));
            }
        }
        if (h->ndamp) {
            DG_ALLOC(h->damp_list, sizeof(int) * list.size());
            DG_ALLOC(h->damp_q0, sizeof(double) * list.size() * (size_t)h->nvar * h->n * h->n * h->g.ew);
            e = hipMemcpyAsync(h->damp_list, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, h->s);
            if (e == hipSuccess) e = hipStreamSynchronize(h->s);
            if (e != hipSuccess) {
                (void)hipFree(prim_dev);
                return bail(hip_fail(h, e, "damping list upload"));
            }
        }
    }
#undef DG_ALLOC

    StepBlock sb0{};
    e = hipMemcpyAsync(h->sb, &sb0, sizeof sb0, hipMemcpyHostToDevice, h->s);
    // padding slots of the tiled layout stay zero in every state array the
    // library writes (the stage kernels skip them, combinations keep zeros)
    if (e == hipSuccess) e = hipMemsetAsync(u0_dev, 0, state_bytes, h->s);
    if (e == hipSuccess) e = hipMemsetAsync(h->ws1, 0, state_bytes, h->s);
    if (e == hipSuccess) e = hipMemsetAsync(h->ws2, 0, state_bytes, h->s);
    if (e == hipSuccess && h->kbuf) e = hipMemsetAsync(h->kbuf, 0, state_bytes * (size_t)h->tab.s, h->s);
    if (e == hipSuccess && h->dev) e = hipMemsetAsync(h->eq, 0, state_bytes, h->s);
    if (e == hipSuccess && h->dev) e = hipMemsetAsync(h->leq, 0, state_bytes, h->s);
    if (e == hipSuccess && h->dev)
        e = hipMemsetAsync(h->eqtr, 0, sizeof(float) * (size_t)dgk::eq_trace_entries(h->n, h->g), h->s);
    if (e == hipSuccess) e = hipMemcpyAsync(prim_dev, prim_nodes_host, prim_bytes, hipMemcpyHostToDevice, h->s);
    if (e == hipSuccess) e = dgk::launch_project(h->n, h->nvar, h->g, prim_dev, u0_dev, h->s);
    // the positivity limiter acts on the projected initial state too
    if (e == hipSuccess && cfg->positivity)
        e = dgk::launch_troubled(h->n, h->nvar, h->g, u0_dev, nullptr, 0.0, 2, 1, nullptr, nullptr, nullptr, nullptr, 1,
                                 nullptr, h->s);
    if (e == hipSuccess) e = hipMemcpyAsync(h->u0, u0_dev, state_bytes, hipMemcpyDeviceToDevice, h->s);
    if (e == hipSuccess) e = hipStreamSynchronize(h->s);
    if (e != hipSuccess) {
        (void)hipFree(prim_dev);
        return bail(hip_fail(h, e, "dg_init projection"));
    }
    if (h->dev) {
        // Deviation form: project the equilibrium (same projection kernel as
        // the state), evaluate L(u_eq) once with the FP64 stage kernel (no
        // planet, exterior state = u_eq) and keep it in FP64, tabulate u_eq's
        // edge traces; the caller's u0_dev and the fixed exterior state become
        // deviations u0 - u_eq.
        std::vector<double> peq;
        equilibrium_prim(cfg, &peq);
        const long long N = (long long)h->nvar * h->n * h->n * h->g.slots;
        Geo g0 = h->g;
        g0.q = 0.0;
        e = hipMemcpyAsync(prim_dev, peq.data(), sizeof(double) * peq.size(), hipMemcpyHostToDevice, h->s);
        if (e == hipSuccess) e = dgk::launch_project(h->n, h->nvar, h->g, prim_dev, h->eq, h->s);
        if (e == hipSuccess) e = dgk::launch_set_coeffs(h->sc_rhs, g0, 0.0, 0.0, 0.0, 1.0, h->s);
        if (e == hipSuccess) e = dgk::launch_stage(h->n, g0, h->eq, nullptr, h->eq, h->leq, h->sc_rhs, false, nullptr, h->s);
        if (e == hipSuccess) e = dgk::launch_eq_traces(h->n, h->g, h->eq, h->eqtr, h->s);
        if (e == hipSuccess) e = dgk::launch_add_state(u0_dev, h->eq, u0_dev, -1.0, N, h->s);
        if (e == hipSuccess) e = hipMemcpyAsync(h->du0, u0_dev, state_bytes, hipMemcpyDeviceToDevice, h->s);
        if (e == hipSuccess) e = hipStreamSynchronize(h->s);  // peq lives until here
        if (e != hipSuccess) {
            (void)hipFree(prim_dev);
            return bail(hip_fail(h, e, "dg_init equilibrium"));
        }
    }
    (void)hipFree(prim_dev);
    // damping targets from u0, which is fixed from here on
    if (h->ndamp) {
        e = dgk::launch_damp_prep(h->n, h->g, h->u0, h->damp_list, h->ndamp, h->damp_q0, h->s);
        if (e != hipSuccess) return bail(hip_fail(h, e, "damping targets"));
    }
    // feature scales: RMS of the initial element means of each variable
    {
        // the means of u0, gathered into [v][e] in the stage workspace
        std::vector<double> means((size_t)h->E);
        e = dgk::launch_means(h->n, h->nvar, h->g, h->u0, h->ws1, h->s);
        if (e == hipSuccess) e = hipStreamSynchronize(h->s);
        for (int v = 0; v < h->nvar && e == hipSuccess; ++v) {
            e = hipMemcpy(means.data(), h->ws1 + (size_t)v * h->E, sizeof(double) * h->E, hipMemcpyDeviceToHost);
            double ss = 0.0;
            for (double m : means) ss += m * m;
            h->scale_host[v] = std::sqrt(ss / (double)h->E);
        }
        if (e == hipSuccess) e = hipMemcpy(h->scale_dev, h->scale_host, sizeof(double) * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(h->mlp, 0, sizeof(float) * 3 * (size_t)dgk::mlp_nparam());
        if (e != hipSuccess) return bail(hip_fail(h, e, "dg_init feature scales"));
    }
    *out = h;
    return DG_OK;
}

int dg_rhs(dg_handle* h, double t, const double* u_dev, double* rhs_dev) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    if (!u_dev || !rhs_dev || u_dev == rhs_dev) return fail(h, DG_EINVAL, "u_dev and rhs_dev must be distinct device arrays");
    DG_HIP(h, dgk::launch_set_coeffs(h->sc_rhs, h->g, t, 0.0, 0.0, 1.0, h->s), "dg_rhs coefficients");
    DG_HIP(h, h->dev ? dgk::launch_stage_dev(h->n, h->g, u_dev, nullptr, h->du0, h->leq, h->eqtr, rhs_dev, h->sc_rhs,
                                             h->s)
                     : dgk::launch_stage(h->n, h->g, u_dev, nullptr, h->u0, rhs_dev, h->sc_rhs, false, nullptr, h->s),
           "dg_rhs stage");
    return DG_OK;
}

// One step (Algorithm 1); with tq_out (FP64 form) the first stage, whose
// input is u^n at t^n, also forms the torque partials of u^n (h->tq_part),
// and the last stage adds them up into *tq_out.
static int rk_step(dg_handle* h, double* u_dev, double* t_dev, double dt_fixed, double* dt_used_dev,
                   double* tq_out) {
    const bool tq = tq_out != nullptr;
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    if (!u_dev || !t_dev) return fail(h, DG_EINVAL, "u_dev and t_dev are required");
    if (!(dt_fixed == dt_fixed)) return fail(h, DG_EINVAL, "dt_fixed is NaN");
    StepBlock* sb = h->sb;
    double* tqp = tq ? h->tq_part : nullptr;
    DG_HIP(h, dgk::launch_dt(h->n, h->g, u_dev, h->eq, h->dt_part, h->bad_part, h->s), "CFL reduction");
    if (h->tab.s > 0) {
        // Butcher form: k_i = L(y_i), y_1 = u^n, y_i = u^n + dt sum_{j<i} a_ij k_j,
        // u^{n+1} = u^n + dt sum_j b_j k_j (no limiter with these tables)
        const int S = h->tab.s;
        const long long N = (long long)h->nvar * h->n * h->n * h->g.slots;
        const double* k[dgk::kMaxStages];
        for (int i = 0; i < S; ++i) k[i] = h->kbuf + (size_t)i * (size_t)N;
        DG_HIP(h, dgk::launch_step_begin_table(h->g, sb, h->tab, h->dt_part, h->bad_part, h->dt_blocks, t_dev,
                                                         dt_fixed, dt_used_dev, h->s), "step begin");
        for (int i = 0; i < S; ++i) {
            const double* y = i == 0 ? u_dev : h->ws1;
            const bool last = i + 1 == S;
            DG_HIP(h, stage(h, y, nullptr, h->kbuf + (size_t)i * (size_t)N, &sb->st[i], false, i == 0 ? tqp : nullptr,
                            nullptr, nullptr, last && i > 0 ? tq_out : nullptr),
                   "stage");
            if (i + 1 < S) {
                DG_HIP(h, dgk::launch_rk_combine(u_dev, k, i + 1, &sb->comb[i + 1][0], h->ws1, N, h->s), "stage state");
            }
        }
        DG_HIP(h, dgk::launch_rk_combine(u_dev, k, S, &sb->comb[0][0], u_dev, N, h->s), "update");
        if (h->cfg.damping)
            DG_HIP(h, dgk::launch_damp(h->n, h->g, u_dev, h->damp_q0, h->eq, h->damp_list, h->ndamp, &sb->st[0], h->s,
                                       h->rev),
                   "damping");
        return DG_OK;
    }
    if (h->cfg.rk == DG_RK_SSP22) {
        DG_HIP(h, dgk::launch_step_begin(h->g, sb, h->dt_part, h->bad_part, h->dt_blocks, t_dev, dt_fixed,
                                                   dt_used_dev, 2, h->s), "step begin");
        DG_HIP(h, stage(h, u_dev, nullptr, h->ws1, &sb->st[0], false, tqp), "stage 1");
        DG_HIP(h, stage(h, h->ws1, u_dev, u_dev, &sb->st[1], false, nullptr, nullptr, nullptr, tq_out), "stage 2");
        if (h->cfg.damping)
            DG_HIP(h, dgk::launch_damp(h->n, h->g, u_dev, h->damp_q0, h->eq, h->damp_list, h->ndamp, &sb->st[0], h->s,
                                       h->rev),
                   "damping");
        return DG_OK;
    }
    DG_HIP(h, dgk::launch_step_begin(h->g, sb, h->dt_part, h->bad_part, h->dt_blocks, t_dev, dt_fixed,
                                               dt_used_dev, 3, h->s), "step begin");
    // the positivity scaling alone (no troubled-cell limiter before it) runs
    // inside the stage kernels
    const bool fuse = h->cfg.positivity && h->cfg.limiter == DG_LIMITER_NONE && !h->dev;
    // with the learned indicator, each stage kernel forms the flags of the
    // state it writes (the network's weights packed once per step)
    dgk::MlpFlags mlpf{};
    const dgk::MlpFlags* mf = nullptr;
    if (h->cfg.limiter == DG_LIMITER_LEARNED) {
        DG_HIP(h, dgk::launch_mlp_pack(h->mlp, h->mlp_pack, h->s), "network weights");
        const float th = (float)h->cfg.mlp_theta;
        mlpf = dgk::MlpFlags{h->mlp_pack, h->scale_dev, h->flags,
                             std::log(th / (1.0f - th))};  // sigmoid(z) > theta  <=>  z > logit(theta)
        mf = &mlpf;
    }
    // with a troubled-cell limiter and the positivity limiter (order 4,
    // adiabatic) each stage kernel marks the tiles that need no positivity
    // scaling, and the pass after the limiter skips them
    unsigned char* ppk = fuse ? nullptr : h->pp_ok;
    DG_HIP(h, stage(h, u_dev, nullptr, h->ws1, &sb->st[0], fuse, tqp, mf, ppk), "stage 1");
    if (!fuse) DG_HIP(h, limit(h, h->ws1, false), "limiter");
    DG_HIP(h, stage(h, h->ws1, u_dev, h->ws2, &sb->st[1], fuse, nullptr, mf, ppk), "stage 2");
    if (!fuse) DG_HIP(h, limit(h, h->ws2, false), "limiter");
    DG_HIP(h, stage(h, h->ws2, u_dev, u_dev, &sb->st[2], fuse, nullptr, mf, ppk, tq_out), "stage 3");
    if (!fuse) DG_HIP(h, limit(h, u_dev, true), "limiter");
    if (h->cfg.damping) {
        DG_HIP(h, dgk::launch_damp(h->n, h->g, u_dev, h->damp_q0, h->eq, h->damp_list, h->ndamp, &sb->st[0], h->s,
                                       h->rev),
               "damping");
        // the damped state gets the positivity scaling too (damped tiles
        // only: the pass read-only skips the tiles marked undamped)
        if (h->cfg.positivity)
            DG_HIP(h, dgk::launch_troubled(h->n, h->nvar, h->g, u_dev, nullptr, 0.0, 2, 1, nullptr, nullptr, nullptr,
                                           nullptr, 1, nullptr, h->s, h->undamped),
                   "positivity after damping");
    }
    return DG_OK;
}

int dg_rk_step(dg_handle* h, double* u_dev, double* t_dev, double dt_fixed, double* dt_used_dev) {
    return rk_step(h, u_dev, t_dev, dt_fixed, dt_used_dev, nullptr);
}

int dg_rk_step_torque(dg_handle* h, double* u_dev, double* t_dev, double dt_fixed, double* dt_used_dev,
                      double* torque_dev) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    if (!u_dev || !t_dev || !torque_dev) return fail(h, DG_EINVAL, "u_dev, t_dev and torque_dev are required");
    // the deviation form's stage kernel has no torque terms, and the stage
    // kernels with the positivity scaling fused do not take them (registers):
    // there the two calls run one after the other
    if (h->dev || (h->cfg.positivity && h->cfg.limiter == DG_LIMITER_NONE)) {
        const int rc = dg_torque(h, 0.0, t_dev, u_dev, torque_dev);
        return rc != DG_OK ? rc : rk_step(h, u_dev, t_dev, dt_fixed, dt_used_dev, nullptr);
    }
    const int rc = rk_step(h, u_dev, t_dev, dt_fixed, dt_used_dev, torque_dev);
    if (rc != DG_OK) return rc;
    // a one-stage Butcher table has no later stage to add the partials up
    if (h->tab.s == 1) DG_HIP(h, dgk::launch_torque_final(h->g, h->tq_part, torque_dev, h->s), "torque sum");
    return DG_OK;
}

int dg_torque(dg_handle* h, double t, const double* t_dev, const double* u_dev, double* torque_dev) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    if (!u_dev || !torque_dev) return fail(h, DG_EINVAL, "u_dev and torque_dev are required");
    DG_HIP(h, dgk::launch_torque(h->n, h->g, t, t_dev, u_dev, h->eq, h->tq_part, torque_dev, h->s), "torque");
    return DG_OK;
}

int dg_torque_noalloc(const dg_config* cfg, double t, const double* t_dev, const double* u_dev, double* torque_dev,
                      void* hip_stream) {
    std::string why;
    const int rc = validate(cfg, &why);
    if (rc != DG_OK) return fail(nullptr, rc, why);
    if (cfg->precision != DG_PRECISION_FP64)
        return fail(nullptr, DG_EUNSUPPORTED, "dg_torque_noalloc takes full FP64 states (precision DG_PRECISION_FP64)");
    Geo g;
    make_geo(cfg, &g);
    const int nb = dgk::torque_partials(g);
    if (nb > kNoAllocPartials)
        return fail(nullptr, DG_EUNSUPPORTED,
                    "dg_torque_noalloc: the grid needs " + std::to_string(nb) + " partial sums, the static scratch holds " +
                        std::to_string(kNoAllocPartials) + " (one per tile of 64 / order elements)");
    if (!u_dev || !torque_dev) return fail(nullptr, DG_EINVAL, "u_dev and torque_dev are required");
    double* part = nullptr;
    hipError_t e = scratch_of_current_device(&part);
    if (e != hipSuccess) return fail(nullptr, DG_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
    e = dgk::launch_torque(cfg->order, g, t, t_dev, u_dev, nullptr, part, torque_dev, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, DG_EHIP, std::string("torque: ") + hipGetErrorString(e));
    return DG_OK;
}

int dg_troubled(dg_handle* h, double* u_dev, int apply, unsigned char* flag_dev, unsigned char* changed_dev,
                float* sensor_dev) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    if (!u_dev) return fail(h, DG_EINVAL, "NULL state");
    if (h->dev) return fail(h, DG_EUNSUPPORTED, "the limiter runs on the FP64 form");
    DG_HIP(h, dgk::launch_troubled(h->n, h->nvar, h->g, u_dev, h->u0, h->cfg.limiter_s0, 0, apply ? 1 : 0, nullptr,
                                   flag_dev, changed_dev, sensor_dev, 0, nullptr, h->s),
           "troubled cells");
    return DG_OK;
}

int dg_positivity(dg_handle* h, double* u_dev, unsigned char* changed_dev, double* theta_dev) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    if (!u_dev) return fail(h, DG_EINVAL, "NULL state");
    if (h->dev) return fail(h, DG_EUNSUPPORTED, "the limiter runs on the FP64 form");
    DG_HIP(h, dgk::launch_troubled(h->n, h->nvar, h->g, u_dev, nullptr, 0.0, 2, 1, nullptr, nullptr, changed_dev,
                                   nullptr, 1, theta_dev, h->s),
           "positivity limiter");
    return DG_OK;
}

int dg_capture(dg_handle* h, unsigned short* feat_dev, unsigned char* flag_dev, unsigned char* label_dev,
               unsigned char* mlp_flag_dev) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    if (h->cfg.limiter == DG_LIMITER_NONE) return fail(h, DG_EINVAL, "capture needs a configured limiter");
    if (feat_dev && !(h->n == 4 && h->nvar == 4)) return fail(h, DG_EUNSUPPORTED, "features need order 4 and nvar 4");
    h->cap = true;
    h->cap_feat = feat_dev;
    h->cap_flag = flag_dev;
    h->cap_label = label_dev;
    h->cap_mlp = mlp_flag_dev;
    return DG_OK;
}

int dg_mlp_feature_scales(dg_handle* h, double* scales_host) {
    if (!h || !scales_host) return fail(h, DG_EINVAL, "NULL argument");
    for (int v = 0; v < h->nvar; ++v) scales_host[v] = h->scale_host[v];
    return DG_OK;
}

int dg_mlp_features(dg_handle* h, const double* u_dev, unsigned short* feat_dev) {
    if (!h || !u_dev || !feat_dev) return fail(h, DG_EINVAL, "NULL argument");
    if (!(h->n == 4 && h->nvar == 4)) return fail(h, DG_EUNSUPPORTED, "features need order 4 and nvar 4");
    DG_HIP(h, dgk::launch_features(h->n, h->nvar, h->g, u_dev, h->scale_dev, feat_dev, h->s), "features");
    return DG_OK;
}

int dg_mlp_params(dg_handle* h, const float* set_host, float* get_host) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    const size_t np = (size_t)dgk::mlp_nparam();
    if (set_host) {
        DG_HIP(h, hipStreamSynchronize(h->s), "sync");
        DG_HIP(h, hipMemcpy(h->mlp, set_host, sizeof(float) * np, hipMemcpyHostToDevice), "set params");
        DG_HIP(h, hipMemset(h->mlp + np, 0, sizeof(float) * 2 * np), "reset moments");
        h->adam_t = 0;
    }
    if (get_host) {
        DG_HIP(h, hipStreamSynchronize(h->s), "sync");
        DG_HIP(h, hipMemcpy(get_host, h->mlp, sizeof(float) * np, hipMemcpyDeviceToHost), "get params");
    }
    return DG_OK;
}

int dg_mlp_forward(dg_handle* h, const unsigned short* feat_dev, long n, float* logit_dev) {
    if (!h || !feat_dev || !logit_dev || n < 0) return fail(h, DG_EINVAL, "bad argument");
    if (n == 0) return DG_OK;
    DG_HIP(h, dgk::launch_mlp_forward(feat_dev, n, h->mlp, logit_dev, nullptr, nullptr, nullptr, 0.f, h->s), "forward");
    return DG_OK;
}

int dg_mlp_train_step(dg_handle* h, const unsigned short* feat_dev, const float* label_dev, long n, float pos_weight,
                      float lr, float* loss_dev, float* grad_dev) {
    if (!h || !feat_dev || !label_dev || n <= 0) return fail(h, DG_EINVAL, "bad argument");
    const long long nb = dgk::mlp_delta_blocks(n);
    const size_t np = (size_t)dgk::mlp_nparam();
    if (n > h->tr_cap) {
        DG_HIP(h, hipStreamSynchronize(h->s), "sync");
        (void)hipFree(h->tr_ws);
        h->tr_ws = nullptr;
        const size_t need = (size_t)n * (1 + 32 + 32 + 1 + 32 + 32) + (size_t)nb + np;
        hipError_t e = hipMalloc((void**)&h->tr_ws, sizeof(float) * need);
        if (e != hipSuccess) {
            h->tr_cap = 0;
            return fail(h, DG_ENOMEM, "training workspace");
        }
        h->tr_cap = n;
    }
    float* z = h->tr_ws;
    float* h1 = z + n;
    float* h2 = h1 + (size_t)n * 32;
    float* dz = h2 + (size_t)n * 32;
    float* d1 = dz + n;
    float* d2 = d1 + (size_t)n * 32;
    float* lp = d2 + (size_t)n * 32;
    float* grad = grad_dev ? grad_dev : lp + nb;
    DG_HIP(h, dgk::launch_mlp_forward(feat_dev, n, h->mlp, z, h1, h2, nullptr, 0.f, h->s), "forward");
    DG_HIP(h, dgk::launch_mlp_backward(feat_dev, label_dev, n, pos_weight, h->mlp, z, h1, h2, dz, d1, d2, lp, grad, h->s),
           "backward");
    if (lr > 0.f) ++h->adam_t;
    DG_HIP(h, dgk::launch_mlp_adam(grad, lp, (int)nb, h->mlp, h->mlp + np, h->mlp + 2 * np, h->adam_t, lr, 0.9f, 0.999f,
                                   1e-8f, loss_dev, h->s),
           "adam");
    return DG_OK;
}

int dg_full_state(dg_handle* h, const double* dev_dev, double* full_dev) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    if (!dev_dev || !full_dev) return fail(h, DG_EINVAL, "NULL state");
    const long long ns = (long long)h->nvar * h->n * h->n * h->g.slots;
    if (h->dev) {
        DG_HIP(h, dgk::launch_add_state(h->eq, dev_dev, full_dev, 1.0, ns, h->s), "full state");
    } else if (dev_dev != full_dev) {
        DG_HIP(h, hipMemcpyAsync(full_dev, dev_dev, sizeof(double) * ns, hipMemcpyDeviceToDevice, h->s), "copy");
    }
    return DG_OK;
}

int dg_sync(dg_handle* h) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    DG_HIP(h, hipStreamSynchronize(h->s), "hipStreamSynchronize");
    unsigned int flags = 0;
    DG_HIP(h, hipMemcpy(&flags, &h->sb->flags, sizeof flags, hipMemcpyDeviceToHost), "flag read");
    if (flags) {
        const unsigned int zero = 0;
        DG_HIP(h, hipMemcpy(&h->sb->flags, &zero, sizeof zero, hipMemcpyHostToDevice), "flag reset");
        return fail(h, DG_ENONFINITE, "non-finite or non-positive density mean detected");
    }
    return DG_OK;
}

int dg_profile_begin(dg_handle* h) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    DG_HIP(h, hipStreamSynchronize(h->s), "hipStreamSynchronize");
    drop_events(h);
    h->prof = true;
    return DG_OK;
}

int dg_profile_end(dg_handle* h, double* stage_ms, int* stage_launches) {
    if (!h) return fail(nullptr, DG_EINVAL, "NULL handle");
    h->prof = false;
    double tot = 0.0;
    for (size_t k = 0; k + 1 < h->ev.size(); k += 2) {
        DG_HIP(h, hipEventSynchronize(h->ev[k + 1]), "hipEventSynchronize");
        float ms = 0.0f;
        DG_HIP(h, hipEventElapsedTime(&ms, h->ev[k], h->ev[k + 1]), "hipEventElapsedTime");
        tot += ms;
    }
    if (stage_ms) *stage_ms = tot;
    if (stage_launches) *stage_launches = (int)(h->ev.size() / 2);
    drop_events(h);
    return DG_OK;
}

int dg_free(dg_handle* h) {
    if (!h) return DG_OK;
    (void)hipStreamSynchronize(h->s);
    release(h);
    delete h;
    return DG_OK;
}

const char* dg_last_error(const dg_handle* h) { return h ? h->err.c_str() : g_err.c_str(); }

}  // extern "C"
