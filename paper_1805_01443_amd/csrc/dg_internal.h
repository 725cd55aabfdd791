// Internal structures shared by the C-ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgk {

constexpr int kMaxN = 5;  // orders 2..5 (P1..P4)

// State layout (every state array of a handle): elements are grouped in
// tiles of EW = 64 / n consecutive elements of one row (n = order), tile
// t = j * tiles_x + i / EW, slot s = i % EW; inside a tile the entries are
// ordered [v][b][a][s] for mode (a, b) of variable v.  So the n lanes of one
// element that hold its mode rows a = 0..n-1 read, for fixed (v, b), one
// contiguous run of n * EW doubles with the other elements of the tile.
// Slots past the end of a row are padding (never read as neighbours).
constexpr int tile_width(int n) { return 64 / n; }

// Mesh, closure and gravity parameters.
struct Geo {
    int nx, ny;
    long long E;
    int ew;            // elements per tile
    int tiles_x;       // tiles per row
    long long slots;   // tiles_x * ny * ew: elements of the padded layout
    double x0, y0, dx, dy;
    double rdx2, rdy2; // 2/dx, 2/dy
    double idx, idy;   // 1/dx, 1/dy
    int closure, bc, star;
    double cs2;        // isothermal c_s^2
    double cs;         // isothermal c_s
    double rc2, irc;   // r_core^2, 1 / r_core
    double h2gm;       // h^2 GM (locally isothermal)
    double gamma;
    double gm, r_core, rc3inv;  // GM / r_core^3
    double q, eps2;
    double gm_h, rc3inv_h, q_h; // gm, rc3inv, q times dx / 2 (the stage kernel's x projection)
    double rp, phi0, omp;       // planet orbit, Omega_p
    // damping
    int damping;
    double rd_in, rd_out, rb_in, rb_out, td_in, td_out;
    double irw_in, irw_out;     // 1 / (rb - rd) of each zone
    double cfl_fac;             // C / (2 N_p + 1)
    double pp_eps;              // positivity limiter: floor of eps
    double sigma0;              // deviation form: equilibrium Sigma0
    int flux;                   // 0 Rusanov, 1 HLLC (adiabatic closure)
};

// Index (in entries) of mode (0, 0) of variable 0 of element (i, j) in the
// tiled layout, and the offset of mode (a, b) of variable v from it.
template <int N, int NV>
__device__ __forceinline__ unsigned tiled_base(const Geo& g, int i, int j) {
    constexpr int EW = tile_width(N);
    const int ti = i / EW;
    return (unsigned)(j * g.tiles_x + ti) * (unsigned)(NV * N * N * EW) + (unsigned)(i - ti * EW);
}
template <int N>
__device__ __forceinline__ constexpr unsigned mode_off(int v, int a, int b) {
    return (unsigned)(((v * N + b) * N + a) * tile_width(N));
}

// Per-stage coefficients: out = a0 * u^n + a1 * u + a2 * L(u, t)
struct StageCoeffs {
    double t;       // stage time
    double xp, yp;  // planet position at t
    double a0, a1, a2;
    double dt;      // step size (damping)
    double pad;
};

constexpr int kMaxStages = 6;

// Butcher table (row-major A, s <= kMaxStages), passed by value
struct RKTable {
    int s;
    int pad;
    double A[kMaxStages * kMaxStages];
    double b[kMaxStages];
    double c[kMaxStages];
};

// Device-resident per-step block written by the step-begin kernels.
// SSP(3,3) uses st[0..2] as Shu-Osher stage coefficients; a Butcher table
// uses st[i] for k_i = L(y_i) (a0 = a1 = 0, a2 = 1), comb[i][j] = dt a_ij for
// the stage states and comb[0][j] = dt b_j for the update.
struct StepBlock {
    StageCoeffs st[kMaxStages];
    double comb[kMaxStages][kMaxStages];
    unsigned int flags;             // bit 0: non-finite / non-positive mean seen
    unsigned int pad;
};

// launchers (all asynchronous on `s`)
hipError_t launch_project(int n, int nvar, const Geo& g, const double* prim_dev, double* u_dev,
                          hipStream_t s);
// The learned indicator's flags of a stage's new rows (order 4, adiabatic):
// flags[e] = logit > zthr, features u_vm / (|u_v00| + scale_v), weights from
// launch_mlp_pack.
struct MlpFlags {
    const void* pack;
    const double* scale;
    unsigned char* flags;
    float zthr;
};
// pp: the positivity scaling fused into the stage (after the combination);
// tq_part (optional, not with pp; a stage whose input u is the state at the
// stage time): also the torque of eq. (5) on u, one partial per tile
// (torque_partials doubles), for launch_torque_final; mf (optional, order 4
// adiabatic, not with pp): also the learned indicator's flags of out; pp_ok
// (optional, order 4 adiabatic, not with pp): per tile, 1 if no element of
// out needs the positivity scaling (for launch_troubled)
// rev: the tiles of each XCD's band in reverse order (stage launches
// alternate it; the results do not depend on it).  tq_sum, tq_out: the
// torque partials of an earlier first stage (tq_part there) added up into
// *tq_out by one more block, with the bits of launch_torque_final.
hipError_t launch_stage(int n, const Geo& g, const double* u, const double* un, const double* u0,
                        double* out, const StageCoeffs* sc, bool pp, double* tq_part, hipStream_t s,
                        const MlpFlags* mf = nullptr, unsigned char* pp_ok = nullptr, bool rev = false,
                        const double* tq_sum = nullptr, double* tq_out = nullptr);
hipError_t launch_set_coeffs(StageCoeffs* sc, const Geo& g, double t, double a0, double a1,
                             double a2, hipStream_t s);
// CFL step per element; per-block minimum into dt_part[block] and a per-block
// flag (non-finite or non-positive mean) into bad_part[block]
hipError_t launch_dt(int n, const Geo& g, const double* u, const double* eq, double* dt_part,
                     unsigned int* bad_part, hipStream_t s);
int dt_blocks(const Geo& g);
// The step-begin kernels reduce the CFL partials (dt = dt_fixed if > 0, else
// their minimum), OR the flags into sb->flags and write the stage data.
hipError_t launch_step_begin_table(const Geo& g, StepBlock* sb, const RKTable& tab, const double* dt_part,
                                  const unsigned int* bad_part, int nblk, double* t_dev, double dt_fixed,
                                  double* dt_used, hipStream_t s);
// out = base + sum_{j < nk} coef[j] k[j] (coef: device array); out may alias base
hipError_t launch_rk_combine(const double* base, const double* const* k, int nk, const double* coef,
                             double* out, long long n, hipStream_t s);
// nst = 3: SSP(3,3), nst = 2: SSP(2,2), Shu-Osher coefficients in sb->st
hipError_t launch_step_begin(const Geo& g, StepBlock* sb, const double* dt_part, const unsigned int* bad_part,
                             int nblk, double* t_dev, double dt_fixed, double* dt_used_dev, int nst, hipStream_t s);
// damping targets of the listed tiles from u0 (once), q0: nlist NV n n EW doubles
hipError_t launch_damp_prep(int n, const Geo& g, const double* u0, const int* list, int nlist, double* q0,
                            hipStream_t s);
// rev: the list from its end
hipError_t launch_damp(int n, const Geo& g, double* u, const double* q0, const double* eq, const int* list,
                       int nlist, const StageCoeffs* sc, hipStream_t s, bool rev = false);
// torque of eq. (5): one partial per tile into partials (torque_partials
// doubles), then their sum in a fixed order into *out
hipError_t launch_torque(int n, const Geo& g, double t, const double* t_dev, const double* u, const double* eq,
                         double* partials, double* out, hipStream_t s);
// the fixed-order sum alone, of partials a stage kernel wrote
hipError_t launch_torque_final(const Geo& g, const double* partials, double* out, hipStream_t s);
// deviation form: leq = L(u_eq) (FP64), eqtr = u_eq's edge traces (FP32,
// eq_trace_entries floats, written by launch_eq_traces)
hipError_t launch_stage_dev(int n, const Geo& g, const double* du, const double* dun, const double* du0,
                            const double* leq, const float* eqtr, double* out, const StageCoeffs* sc,
                            hipStream_t s, bool rev = false);
long long eq_trace_entries(int n, const Geo& g);
hipError_t launch_eq_traces(int n, const Geo& g, const double* eq, float* eqtr, hipStream_t s);
hipError_t launch_add_state(const double* a, const double* b, double* out, double sign, long long n,
                            hipStream_t s);
int torque_partials(const Geo& g);

// troubled cells and the learned indicator
// means of every variable into out[v * E + e] (contiguous), from a state array
hipError_t launch_means(int n, int nvar, const Geo& g, const double* u, double* out, hipStream_t s);
// pp_ok (optional, with pp and no changed_out / theta_out): the stage
// kernel's per-tile marks; elements that minmod changes clear their tile's
// mark, and the positivity pass skips the tiles still marked
hipError_t launch_troubled(int n, int nvar, const Geo& g, double* u, const double* u0, double s0, int mode, int apply,
                           const unsigned char* flag_in, unsigned char* flag_out, unsigned char* changed_out,
                           float* sensor_out, int pp, double* theta_out, hipStream_t s,
                           unsigned char* pp_ok = nullptr);
hipError_t launch_features(int n, int nvar, const Geo& g, const double* u, const double* scale, unsigned short* f,
                           hipStream_t s);
hipError_t launch_mlp_forward(const unsigned short* x, long long n, const float* par, float* z, float* h1, float* h2,
                              unsigned char* flags, float zthr, hipStream_t s);
// the network's weights in per-lane fragment form (mlp_pack_bytes), for the
// stage kernel that forms the learned indicator's flags
hipError_t launch_mlp_pack(const float* par, void* pack, hipStream_t s);
int mlp_pack_bytes();
int mlp_delta_blocks(long long n);
int mlp_nparam();
hipError_t launch_mlp_backward(const unsigned short* x, const float* y, long long n, float pos_weight,
                               const float* par, const float* z, const float* h1, const float* h2, float* dz,
                               float* d1, float* d2, float* loss_part, float* grad, hipStream_t s);
hipError_t launch_mlp_adam(const float* grad, const float* loss_part, int nblk, float* par, float* m, float* v,
                           long long t, float lr, float b1, float b2, float eps, float* loss_out, hipStream_t s);

}  // namespace dgk
