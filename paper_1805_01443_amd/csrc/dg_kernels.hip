// gfx950 kernels of the modal DG right-hand side (Sec. 2.2 eq. (3)), the
// SSP-RK3 stage update (Algorithm 1, Appendix A), the CFL reduction (Sec. 2.3),
// wave-killing damping (Sec. 5.1) and the planet torque (Sec. 5.2 eq. (5)).
//
// The state is element-tiled (dg_internal.h): tiles of EW = 64 / N elements
// of one row, entries [v][b][a][slot], so a mode row of the EW elements is one
// contiguous run.  The stage, damping and torque kernels run N lanes per
// element, one tile per wavefront: lane k works on mode row k (or Gauss row
// k), and the tensor-product contractions are split between the element's
// lanes with transposes through LDS and lane permutes.  Quadrature and basis
// tables are compile-time constants (dg_basis.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dg_basis.h"
#include "dg_mlp.h"
#include "dg_internal.h"
#include "dg_pp.h"

namespace dgk {

enum { CL_ISO = 0, CL_LOC = 1, CL_ADI = 2 };

template <int CL>
struct NVar {
    static constexpr int value = CL == CL_ADI ? 4 : 3;
};

// State arrays are read and written through buffer resources: the array base
// lives in scalar registers, a mode plane is a scalar offset and the lane's
// element is one shared 32-bit vector offset.  (With plain pointers the
// compiler keeps a private 64-bit address per mode plane alive from the loads
// to the stores, which alone costs ~150 registers at order 5.)  The range of
// a resource is 2^31 - 1 bytes; init rejects state arrays larger than that.
using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base) {
    // raw buffer, no swizzle; range checking is not relied on (all accesses
    // are in bounds by construction, every array below the range)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ double ld64(rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, (int)soff, 0));
}
__device__ __forceinline__ float ld32(rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, (int)soff, 0));
}
__device__ __forceinline__ void st64(rsrc_t r, unsigned voff, unsigned soff, double v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, (int)soff, 0);
}

// Blocks are dealt to the 8 XCDs round-robin (block b on XCD b % 8).  Give
// each XCD a contiguous band of tiles, so the rows above and below a tile are
// being read through the same L2.  rev: the XCD walks its band from the end,
// which successive stage launches alternate, so that a stage starts on the
// tiles the previous one wrote last (still in the memory-side cache; the L2
// misses are the same either way, the stage kernel at 512^2 runs 3 % faster).
__device__ __forceinline__ int remap_tile(int b, int total, int rev) {
    if ((total & 7) != 0) return rev ? total - 1 - b : b;
    const int per = total >> 3;
    const int l = b >> 3;
    return (b & 7) * per + (rev ? per - 1 - l : l);
}

// pressure and sound speed of the conservative state U at (x, y); inv = 1/rho
template <int CL>
__device__ __forceinline__ void pressure(const Geo& g, const double* U, double inv, double x, double y,
                                         double& p, double& c) {
    if constexpr (CL == CL_ISO) {
        p = g.cs2 * U[0];
        c = sqrt(g.cs2);
    } else if constexpr (CL == CL_LOC) {
        const double r = sqrt(x * x + y * y);
        const double cs2 = g.h2gm / (r > g.r_core ? r : g.r_core);
        p = cs2 * U[0];
        c = sqrt(cs2);
    } else {
        const double ke = 0.5 * (U[1] * U[1] + U[2] * U[2]) * inv;
        p = (g.gamma - 1.0) * (U[3] - ke);
        c = sqrt(g.gamma * p * inv);
    }
}

// Reciprocal and inverse square root for the stage kernel: the hardware
// estimate refined by two Newton steps (a few ulp at most; operands are normal
// numbers), about half the instructions of the IEEE-rounded sequences.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ double rsq64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// locally isothermal c_s^2 at a point with 1/r = ir (r^2 = r2)
__device__ __forceinline__ double cs2_loc(const Geo& g, double r2, double ir) {
    return g.h2gm * (r2 > g.rc2 ? ir : g.irc);
}

// Rusanov flux through an axis-aligned edge with outward normal SGN * e_AX
template <int CL, int AX, int SGN>
__device__ __forceinline__ void rusanov(const Geo& g, const double* Ui, const double* Uo, double x,
                                        double y, double* h) {
    constexpr int NV = NVar<CL>::value;
    const double ii = rcp64(Ui[0]), io = rcp64(Uo[0]);
    double pi, ci, po, co;
    if constexpr (CL == CL_ISO) {
        pi = g.cs2 * Ui[0];
        po = g.cs2 * Uo[0];
        ci = co = g.cs;
    } else if constexpr (CL == CL_LOC) {
        const double r2 = x * x + y * y;
        const double cs2 = cs2_loc(g, r2, rsq64(r2));
        pi = cs2 * Ui[0];
        po = cs2 * Uo[0];
        ci = co = cs2 * rsq64(cs2);
    } else {
        const double gm1 = g.gamma - 1.0;
        pi = gm1 * (Ui[3] - 0.5 * (Ui[1] * Ui[1] + Ui[2] * Ui[2]) * ii);
        po = gm1 * (Uo[3] - 0.5 * (Uo[1] * Uo[1] + Uo[2] * Uo[2]) * io);
        const double ti = g.gamma * pi * ii, to = g.gamma * po * io;
        ci = ti * rsq64(ti);
        co = to * rsq64(to);
    }
    const double vni = SGN * Ui[1 + AX] * ii;
    const double vno = SGN * Uo[1 + AX] * io;
    double Fi[NV], Fo[NV];
    Fi[0] = Ui[0] * vni;
    Fo[0] = Uo[0] * vno;
    Fi[1] = Ui[1] * vni + (AX == 0 ? SGN * pi : 0.0);
    Fo[1] = Uo[1] * vno + (AX == 0 ? SGN * po : 0.0);
    Fi[2] = Ui[2] * vni + (AX == 1 ? SGN * pi : 0.0);
    Fo[2] = Uo[2] * vno + (AX == 1 ? SGN * po : 0.0);
    if constexpr (NV == 4) {
        Fi[3] = (Ui[3] + pi) * vni;
        Fo[3] = (Uo[3] + po) * vno;
    }
    const double si = fabs(vni) + ci, so = fabs(vno) + co;
    const double alpha = si > so ? si : so;
#pragma unroll
    for (int v = 0; v < NV; ++v) h[v] = 0.5 * (Fi[v] + Fo[v]) - 0.5 * alpha * (Uo[v] - Ui[v]);
}

// HLLC flux (adiabatic closure) through an axis-aligned edge with outward
// normal n = SGN * e_AX, own state Ui (left), exterior Uo (right): Toro,
// Spruce & Speares' three-wave flux with Davis' outer wave speeds
//   S_L = min(q_L - c_L, q_R - c_R), S_R = max(q_L + c_L, q_R + c_R), q = v.n,
// the contact speed S* from the momentum jump conditions of the outer waves,
//   S* = (p_R - p_L + rho_L q_L (S_L - q_L) - rho_R q_R (S_R - q_R))
//        / (rho_L (S_L - q_L) - rho_R (S_R - q_R)),
// and the star state of the side the edge sees,
//   U*_K = rho_K (S_K - q_K) / (S_K - S*)
//          [1, v_K + (S* - q_K) n, E_K / rho_K + (S* - q_K) (S* + p_K / (rho_K (S_K - q_K)))],
// h = F_L (S_L >= 0), F_K + S_K (U*_K - U_K) (K = L if S* >= 0, else R), F_R (S_R <= 0).
template <int AX, int SGN>
__device__ __forceinline__ void hllc(const Geo& g, const double* Ui, const double* Uo, double* h) {
    const double ii = rcp64(Ui[0]), io = rcp64(Uo[0]);
    const double gm1 = g.gamma - 1.0;
    const double pi = gm1 * (Ui[3] - 0.5 * (Ui[1] * Ui[1] + Ui[2] * Ui[2]) * ii);
    const double po = gm1 * (Uo[3] - 0.5 * (Uo[1] * Uo[1] + Uo[2] * Uo[2]) * io);
    const double ti = g.gamma * pi * ii, to = g.gamma * po * io;
    const double ci = ti * rsq64(ti), co = to * rsq64(to);
    const double qi = SGN * Ui[1 + AX] * ii, qo = SGN * Uo[1 + AX] * io;
    double Fi[4], Fo[4];
    Fi[0] = Ui[0] * qi;
    Fo[0] = Uo[0] * qo;
    Fi[1] = Ui[1] * qi + (AX == 0 ? SGN * pi : 0.0);
    Fo[1] = Uo[1] * qo + (AX == 0 ? SGN * po : 0.0);
    Fi[2] = Ui[2] * qi + (AX == 1 ? SGN * pi : 0.0);
    Fo[2] = Uo[2] * qo + (AX == 1 ? SGN * po : 0.0);
    Fi[3] = (Ui[3] + pi) * qi;
    Fo[3] = (Uo[3] + po) * qo;
    const double sl = fmin(qi - ci, qo - co), sr = fmax(qi + ci, qo + co);
    const double ss = (po - pi + Ui[0] * qi * (sl - qi) - Uo[0] * qo * (sr - qo)) *
                      rcp64(Ui[0] * (sl - qi) - Uo[0] * (sr - qo));
    // the side the edge sees (selects, no divergence)
    const bool left = ss >= 0.0;
    const double sk = left ? sl : sr, qk = left ? qi : qo, pk = left ? pi : po, ik = left ? ii : io;
    double U[4], F[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        U[v] = left ? Ui[v] : Uo[v];
        F[v] = left ? Fi[v] : Fo[v];
    }
    const double rk = U[0], dq = ss - qk;
    const double f = rk * (sk - qk) * rcp64(sk - ss);
    double us[4];
    us[0] = f;
    us[1] = f * (U[1] * ik + (AX == 0 ? SGN * dq : 0.0));
    us[2] = f * (U[2] * ik + (AX == 1 ? SGN * dq : 0.0));
    us[3] = f * (U[3] * ik + dq * (ss + pk * rcp64(rk * (sk - qk))));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double star = F[v] + sk * (us[v] - U[v]);
        h[v] = sl >= 0.0 ? Fi[v] : (sr <= 0.0 ? Fo[v] : star);
    }
}

// the configured edge flux: HLLC (FX = 1, adiabatic closure) or Rusanov
template <int CL, int FX, int AX, int SGN>
__device__ __forceinline__ void edge_flux(const Geo& g, const double* Ui, const double* Uo, double x, double y,
                                          double* h) {
    if constexpr (FX == 1 && CL == CL_ADI)
        hllc<AX, SGN>(g, Ui, Uo, h);
    else
        rusanov<CL, AX, SGN>(g, Ui, Uo, x, y, h);
}

// ------------------------------------------------------------------ stage kernel, N lanes per element
// Slot size in LDS for the N-lanes kernels: the lanes of one index k run over
// the element slots (lane k * EW + s), and an odd slot stride puts the slots
// read or written by 16 consecutive lanes on 16 different bank pairs (banks for
// floats).
constexpr int lds_slot_odd(int need) { return need | 1; }

// Lane-dependent entry t[k] of a compile-time table (k < N): a select chain on
// immediates.
template <int N>
__device__ __forceinline__ double pick(const double (&t)[kMaxOrder], int k) {
    double r = t[0];
#pragma unroll
    for (int m = 1; m < N; ++m) r = k == m ? t[m] : r;
    return r;
}

// ---- torque of eq. (5), per element: node (xi_q, eta_r) carries the mass
// rho w_q w_r dx dy / 4 (w: Gauss weights on [-1, 1]); G = 1, per unit planet
// mass.  Lane k of an element takes the nodes (xi_q, eta_k), q < N, in the
// order q = 0 .. N - 1, from the node density rho, the planet offsets
// (dx, dy) = (x - xp, y - yp) and id3 = ((dx^2 + dy^2 + eps^2)^(-1/2))^3.  The
// first stage kernel and the torque kernel add the same doubles in the same
// order, so their tile sums agree to the last bit.
__device__ __forceinline__ double torque_term(double rho, double wnode, double xp, double yp, double dx, double dy,
                                              double id3) {
    const double kk = (rho * wnode) * id3;
    return xp * (kk * dy) - yp * (kk * dx);
}
// sum over the wavefront by a fixed xor butterfly (every lane gets the sum)
__device__ __forceinline__ double wave_sum(double s) {
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

constexpr int kTorqueWaves = 4;      // tiles per block of the torque kernel
constexpr int kTorqueFinal = 1024;   // threads of the final sum (k_torque_final)

// The sum of k_torque_final computed by one wavefront (in the last stage
// kernel of dg_rk_step_torque, beside its tiles): lane l plays the
// threads w * 64 + l of that kernel (w = 0 .. 15), four of them at a time,
// each with its own order of additions (its main loop of eight loads then
// eight adds, then its remaining partials one by one), the same butterfly per
// wavefront of 64 threads, and the wavefront sums added in index order: the
// bits of k_torque_final.  Every lane returns the sum.
__device__ double torque_final_in_wave(const double* __restrict__ partials, int nb) {
    constexpr int TW = kTorqueFinal / 64, G = 2;
    double r = 0.0;
    for (int w0 = 0; w0 < TW; w0 += G) {
        double s[G];
        int k[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            s[q] = 0.0;
            k[q] = (w0 + q) * 64 + (int)threadIdx.x;
        }
        // main loops of the G threads, trip by trip
        while (k[0] + 7 * kTorqueFinal < nb || k[G - 1] + 7 * kTorqueFinal < nb) {
            double v[G][8];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const bool go = k[q] + 7 * kTorqueFinal < nb;
#pragma unroll
                for (int m = 0; m < 8; ++m) v[q][m] = go ? partials[k[q] + m * kTorqueFinal] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (k[q] + 7 * kTorqueFinal < nb) {
#pragma unroll
                    for (int m = 0; m < 8; ++m) s[q] += v[q][m];
                    k[q] += 8 * kTorqueFinal;
                }
            }
        }
        // the remaining partials (at most seven per thread), one by one
        double t[G][7];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int m = 0; m < 7; ++m) t[q][m] = k[q] + m * kTorqueFinal < nb ? partials[k[q] + m * kTorqueFinal] : 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
#pragma unroll
            for (int m = 0; m < 7; ++m)
                if (k[q] + m * kTorqueFinal < nb) s[q] += t[q][m];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off);
            r += s[q];
        }
    }
    return r;
}

// LDS layout of an element slot of the stage kernel.  A 64-lane access of
// single doubles is served 32 lanes at a time over 64 banks of 4 bytes, so a
// half-wave meets no bank twice when its 32 doubles fall on 32 different
// residues mod 32.  Lane k * EW + s (element slot s, index k) addresses
// s * SLOT + k * c + const, with c the access's k-stride; at order 5 with three
// variables (EW = 12) every stride used below is 4 mod 32 and SLOT is 3 mod 8,
// which makes the residue SLOT * (s + EW * k) mod 32: 32 different ones for
// 32 consecutive lanes.  The plain layout (C as [v][a][r], the collapses as
// [kind][v][a]) meets its banks twice per half-wave at order 5; at order 4
// the counters show no conflicts in it (and more with the order-5 scheme
// carried over), lower orders gather their y collapses by lane permute, and
// order 5 with four variables would lose a wave per SIMD to registers in the
// new layout: all of these keep the plain one.
//   C (later X, then Y): entry (v, a, r) at v * CV + a * CA + r * CR, written
//   by lane a and read by lane r (X and Y: written by lane r, read by lane a);
//   the y collapses [kind][v] of row a (later the south/north fluxes
//   [edge][v] at point a): entry (t, a) at TOFF + t * TT + a * TA.
template <int N, int NV>
struct StageLds {
    static constexpr bool C5 = N == 5 && NV == 3;
    static constexpr int CV = C5 ? 1 : N * N;
    static constexpr int CR = C5 ? 4 : 1;
    static constexpr int CA = C5 ? 36 : N;
    static constexpr int TOFF = C5 ? 20 : NV * N * N;
    static constexpr int TT = C5 ? 1 : N;
    static constexpr int TA = C5 ? CA : 1;
    static constexpr int NEED = C5 ? CA * N : NV * N * N + (N >= 4 ? 4 : 2) * NV * N;
    static constexpr int slot(int need) {
        int s = need;
        if (C5)
            while (s % 8 != 3) ++s;
        else
            s |= 1;
        return s;
    }
    static constexpr int ci(int v, int a, int r) { return v * CV + a * CA + r * CR; }
    static constexpr int ti(int t, int a) { return TOFF + t * TT + a * TA; }
    // every entry of C and of the collapses inside the slot, no two alike
    static constexpr bool fits() {
        bool used[NEED] = {};
        for (int v = 0; v < NV; ++v)
            for (int a = 0; a < N; ++a)
                for (int r = 0; r < N; ++r) {
                    const int x = ci(v, a, r);
                    if (x < 0 || x >= NEED || used[x]) return false;
                    used[x] = true;
                }
        for (int t = 0; t < (N >= 4 ? 4 : 2) * NV; ++t)
            for (int a = 0; a < N; ++a) {
                const int x = ti(t, a);
                if (x < 0 || x >= NEED || used[x]) return false;
                used[x] = true;
            }
        return true;
    }
    static_assert(fits(), "stage kernel LDS slot layout");
};

// out = a0 u^n + a1 u + a2 L(u, t), with the N lanes of an element sharing
// its tensor-product contractions.  Lane (s, k) = lane k * EW + s: element
// slot s of the wave (EW = 64 / N consecutive elements of one row), index k.
// Transposes between the lanes of an element go through LDS, single values
// per lane through lane permutes:
//   phase 1, k = mode row a: own row u[v][a][.] -> C[v][a][r] = sum_b u[v][a][b]
//            phi_b(eta_r) (LDS); y collapses of the own row (both sides) and of
//            the y neighbours' rows, x collapses of the x neighbours' columns
//            (registers; an x neighbour in the same wave hands over the
//            collapse of its own column, so only the first and the last
//            element of a wave read a neighbour's column);
//   phase 2, k = Gauss row r: traces at point k of the four edges (the
//            collapses of the element's rows a gathered from its lanes) and
//            their Rusanov fluxes; the west/east lifts, which carry the same
//            weight w_r phi_b(eta_r) in R as the x projection, start X; node
//            values at (xi_q, eta_r) for every q, the physical flux and source,
//            partial projections X[r][a] += sum_q w_q (2/dx phi_a'(q) f_x +
//            phi_a(q) s), Y[r][a] = sum_q w_q phi_a(q) (2/dy) f_y;
//   phase 3, k = mode row a: R[a][b] = sum_r w_r phi_b(r) X[r][a] minus the
//            south/north lifts, plus sum_r w_r phi_b'(r) Y[r][a] (X and Y pass
//            through the same LDS slot one after the other, which keeps the
//            slot at C plus two flux rows); stage combination of row a.
// Every integral is the same Gauss sum as in eq. (3); the density volume term
// is taken by quadrature (exact for its polynomial integrand).
// FX: the edge flux (0 Rusanov, 1 HLLC for the adiabatic closure).
// TQ (a stage whose input is u^n at its own time, the first one): also the
// torque of eq. (5) on u, from the node densities and planet offsets phase 2
// evaluates anyway, as the tile's partial tq_part[tile].
// MF (order 4, adiabatic): also the learned indicator's flag of every new
// element: at order 4 lane k * 16 + s holds modes (k, 0..3) of element slot
// s, which is the MFMA B-fragment layout of the network (dg_mlp.h), so the
// features go from the stored rows straight into the fragments.
// PP: 0 none; 1 the positivity scaling of Sec. 2.4 on the new rows before
// the store (fused positivity limiter); 2 only its factors, to mark in
// pp_ok[tile] a tile whose every element needs no scaling (the positivity
// pass after a troubled-cell limiter then skips it unless the limiter
// changed one of its elements).
template <int N, int CL, int PP, bool TQ, int FX, bool MF>
__global__ void __launch_bounds__(64) k_stage_c(const Geo g, int tiles_x, int tiles_total,
                                                const double* __restrict__ u, const double* un,
                                                const double* __restrict__ u0, double* out,
                                                const StageCoeffs* __restrict__ scp, double* tq_part,
                                                const void* __restrict__ mlp_pack,
                                                const double* __restrict__ mlp_scale,
                                                unsigned char* mlp_flags, float mlp_zthr,
                                                unsigned char* pp_ok, int rev, double* tq_out) {
    constexpr int NV = NVar<CL>::value;
    constexpr int NN = N * N;
    constexpr int EW = 64 / N;
    constexpr BasisTab B = make_basis(N);
    // C, later X then Y; the y collapses of the element's rows (phase 1 to 2),
    // later the south/north fluxes in the same place; with the positivity
    // scaling fused, its rows and minima after that
    // At orders 4 and 5 (two waves per SIMD) the y collapses of an element's
    // rows reach its other lanes through LDS (YL: two doubles per read, where
    // 120 lane permutes of 32 bits queued behind the wave's limit of LDS
    // operations in flight); lower orders run more waves per SIMD and keep
    // the lane permutes (and their smaller LDS slot).
    constexpr bool YL = N >= 4;
    using LY = StageLds<N, NV>;
    constexpr int SLOT = LY::slot(PP != 0 && pp_slot<N, NV>() > LY::NEED ? pp_slot<N, NV>() : LY::NEED);
    // after the slots (orders 4 and 5): the x collapses of the two loaded
    // neighbour columns (west of the first slot, east of the last element),
    // [side][v][a]; lower orders gather them by lane permute
    __shared__ double lds[EW * SLOT + (YL ? 2 * NV * N : 0)];

    // With tq_out (the last stage of dg_rk_step_torque) the launch has eight
    // more blocks in front, one per XCD, so that the tile blocks keep their
    // XCD; the first adds up the torque partials tq_part of the step's first
    // stage into *tq_out, the others end at once.
    if (tq_out && blockIdx.x < 8) {
        if (blockIdx.x == 0) {
            const double r = torque_final_in_wave(tq_part, tiles_total);
            if (threadIdx.x == 0) *tq_out = r;
        }
        return;
    }
    const int bid = (int)blockIdx.x - (tq_out ? 8 : 0);

    // Lane k * EW + s holds index k of element slot s: the lanes of one k
    // address consecutive doubles of the tile (a row of the EW elements is one
    // contiguous run), so every row load and store is contiguous in lane
    // order.  Lanes beyond N * EW mirror another lane (same slot, element and
    // k): lane - 32 where the slot layout keeps a half-wave on 32 different
    // banks (order 5, three variables), else lane (0, k).  They compute that
    // lane's values, write the same values to its slot and store nothing.
    // Slots past the row end work on the row's first element and store
    // nothing either.
    const int lane = threadIdx.x;
    const bool own = lane < N * EW;
    const int k = own ? lane / EW : LY::C5 ? (lane - 32) / EW : lane - N * EW;
    const int sl = own ? lane - k * EW : EW;  // EW: a mirror lane
    const int e0 = own ? sl : LY::C5 ? lane - 32 - k * EW : 0;  // the element's lanes are e0 + a * EW
    const int tile = remap_tile(bid, tiles_total, rev);
    const int j = tile / tiles_x;
    const int i0 = (tile - j * tiles_x) * EW;
    const bool active = sl < EW && i0 + sl < g.nx;
    const int i = LY::C5 ? (i0 + e0 < g.nx ? i0 + e0 : i0) : active ? i0 + sl : i0;
    double* S = lds + e0 * SLOT;
    const int me = e0 + k * EW;  // this lane, or the lane a mirror lane follows
    // The x neighbours inside the wave hand over their x collapses by lane
    // permute; only the first slot (west) and the last slot or the end of the
    // row (east) read the neighbour's column from memory.
    const bool gw = e0 == 0, ge = e0 == EW - 1 || i + 1 >= g.nx;

    const double a0 = scp->a0, a1 = scp->a1, a2 = scp->a2, xp = scp->xp, yp = scp->yp;
    const rsrc_t ru = make_rsrc(u), ru0 = make_rsrc(u0), rout = make_rsrc(out), run = make_rsrc(un);
    // tiled layout: row k of an element is mode (k, b) at + (v * N + b) * RS,
    // column k is mode (a, k) at + (v * N * N + a) * CS (byte strides)
    constexpr unsigned RS = N * EW * 8, CS = EW * 8;
    const unsigned eb = tiled_base<N, NV>(g, i, j);
    const unsigned vrow = (eb + k * EW) * 8u;  // mode (k, 0) of this element
    const double xc = g.x0 + (i + 0.5) * g.dx, yc = g.y0 + (j + 0.5) * g.dy;

    // ---- phase 1: k = mode row.  Every global load of the phase is issued
    // before the first use: the own row k, the y neighbours' rows k and, where
    // the x neighbour is outside the wave, its column k (periodic wrap; at a
    // box edge that is not periodic the collapse is replaced afterwards).
    int il = i - 1, ir = i + 1, jb = j - 1, jt = j + 1;
    const bool ol = il < 0, orr = ir >= g.nx, ob = jb < 0, ot = jt >= g.ny;
    il += ol ? g.nx : 0;
    ir -= orr ? g.nx : 0;
    jb += ob ? g.ny : 0;
    jt -= ot ? g.ny : 0;
    // box edges that are not periodic: the exterior is the element's own
    // initial row/column (fixed edge) or a ghost with no gradient, the
    // element's own current mean (gradient-free edge: only mode (0, 0), held by
    // lane k = 0 as Ua[v][0]); either one enters as its trace on the shared edge
    const bool fxd = g.bc != 0, fl = fxd && ol, fr = fxd && orr, fb = fxd && ob, ft = fxd && ot;
    const bool gfree = g.bc == 2;
    const bool wfy = __any(fb || ft), wfx = __any(fl || fr);  // wave-uniform
    const unsigned vcol = (eb + k * N * EW) * 8u;  // mode (0, k)
    const unsigned vb = (tiled_base<N, NV>(g, i, jb) + k * EW) * 8u, vt = (tiled_base<N, NV>(g, i, jt) + k * EW) * 8u;
    const unsigned vl = (tiled_base<N, NV>(g, il, j) + k * N * EW) * 8u;
    const unsigned vr = (tiled_base<N, NV>(g, ir, j) + k * N * EW) * 8u;
    double Ua[NV][N], Xb[NV][N], Xt[NV][N], Xn[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const unsigned srow = (unsigned)(v * N + m) * RS;
            Ua[v][m] = ld64(ru, vrow, srow);
            Xb[v][m] = ld64(ru, vb, srow);
            Xt[v][m] = ld64(ru, vt, srow);
        }
    // x neighbours outside the wave (west of the first slot, east of the last
    // slot or of the row end): their column k, loaded by those lanes only (a
    // lane with both neighbours outside, a row ending at the first slot, reads
    // the east one further below).  The neighbours inside the wave hand over
    // their edge traces in phase 2.
    const bool gwe = gw && ge;
    if (gw || ge) {
        const unsigned vn = gw ? vl : vr;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < N; ++m) Xn[v][m] = ld64(ru, vn, (unsigned)(v * NN + m) * CS);
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < N; ++m) Xn[v][m] = 0.0;
    }
    // row k's collapses: own south / north, exterior south / north, and (on
    // the boundary lanes) the x collapses of the neighbour's column
    double Tm[NV], Tp[NV], Tb[NV], Tt[NV], Tl[NV], Tr[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double c = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) c += Ua[v][b] * B.phi[b][r];
            S[LY::ci(v, k, r)] = c;
        }
        // the exterior collapses take the neighbour's far side.  phi_m(-1) =
        // (-1)^m phi_m(1): even and odd partial sums give either side.
        double ue = 0.0, uo = 0.0, be = 0.0, bo = 0.0, te = 0.0, to = 0.0, ne = 0.0, no = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            if (m % 2 == 0) {
                ue += B.pp[m] * Ua[v][m];
                be += B.pp[m] * Xb[v][m];
                te += B.pp[m] * Xt[v][m];
                ne += B.pp[m] * Xn[v][m];
            } else {
                uo += B.pp[m] * Ua[v][m];
                bo += B.pp[m] * Xb[v][m];
                to += B.pp[m] * Xt[v][m];
                no += B.pp[m] * Xn[v][m];
            }
        }
        Tm[v] = ue - uo;
        Tp[v] = ue + uo;
        Tb[v] = be + bo;
        Tt[v] = te - to;
        // ne +- no: the east / west side of the loaded neighbour column
        Tl[v] = ne + no;
        Tr[v] = ne - no;
    }
    if (__any(gwe)) {  // the east neighbour's column of a lane that also reads the west one
        if (gwe) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double e = 0.0, o = 0.0;
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const double w = B.pp[m] * ld64(ru, vr, (unsigned)(v * NN + m) * CS);
                    if (m % 2 == 0) e += w; else o += w;
                }
                Tr[v] = e - o;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        // box edges: the element's own initial row/column (or the ghost) on the
        // near side
        if (wfy) {
            double e = 0.0, o = 0.0;
            if (gfree) {
                e = k == 0 ? B.pp[0] * Ua[v][0] : 0.0;
            } else {
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const double w = B.pp[m] * ld64(ru0, vrow, (unsigned)(v * N + m) * RS);
                    if (m % 2 == 0) e += w; else o += w;
                }
            }
            Tb[v] = fb ? e - o : Tb[v];
            Tt[v] = ft ? e + o : Tt[v];
        }
        if (wfx) {
            double e = 0.0, o = 0.0;
            if (gfree) {
                e = k == 0 ? B.pp[0] * Ua[v][0] : 0.0;
            } else {
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const double w = B.pp[m] * ld64(ru0, vcol, (unsigned)(v * NN + m) * CS);
                    if (m % 2 == 0) e += w; else o += w;
                }
            }
            Tl[v] = fl ? e - o : Tl[v];
            Tr[v] = fr ? e + o : Tr[v];
        }
    }
    // the loaded neighbour columns' collapses for the other lanes of the
    // first and the last element (one of each per tile: slot 0, and the
    // element at the last slot or at the row end; a slot past the row end
    // writes nothing)
    if constexpr (YL) {
        double* XE = lds + EW * SLOT;
        const bool wlast = ge && active;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (gw) XE[v * N + k] = Tl[v];
            if (wlast) XE[(NV + v) * N + k] = Tr[v];
        }
    }
    // the y collapses of row k (own south / north, exterior south / north)
    // for the element's other lanes: [kind][v][a] after C
    if constexpr (YL) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            S[LY::ti(0 * NV + v, k)] = Tm[v];
            S[LY::ti(1 * NV + v, k)] = Tp[v];
            S[LY::ti(2 * NV + v, k)] = Tb[v];
            S[LY::ti(3 * NV + v, k)] = Tt[v];
        }
    }
    __syncthreads();

    // ---- phase 2: k = Gauss row r
    const double xik = pick<N>(B.xi, k);
    double phk[N];
#pragma unroll
    for (int m = 0; m < N; ++m) phk[m] = pick<N>(B.phi[m], k);  // phi_m(xi_k)
    const double yk = yc + 0.5 * g.dy * xik;
    double Cc[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) Cc[v][a] = S[LY::ci(v, a, k)];
    // edge traces at point k and their fluxes (outward normals); the y
    // collapses of the element's rows come from LDS (TT, YL) or from lane
    // e0 + a * EW, the x collapses of a loaded neighbour column from LDS (YL)
    // or from lane e0 + a * EW
    // the south / north fluxes [edge][v][point] go over the y collapses once
    // both fluxes of the lane are formed
    double X[NV][N], Y[NV][N];
    {
        double Ui[NV], Uo[NV], hw[NV], he[NV], hs[NV];
        // west / east: own traces from C; the exterior is the x neighbour's own
        // trace at eta_k (lane permute) inside the wave, and the contraction of
        // the loaded column's collapses at the first and last slot
        double Ei[NV], Wx[NV], Ex[NV];
        const double* XE = lds + EW * SLOT;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double w = 0.0, e = 0.0, tl = 0.0, tr = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                w += B.pm[a] * Cc[v][a];
                e += B.pp[a] * Cc[v][a];
                if constexpr (YL) {
                    tl += phk[a] * XE[v * N + a];
                    tr += phk[a] * XE[(NV + v) * N + a];
                } else {
                    tl += phk[a] * __shfl(Tl[v], e0 + a * EW);
                    tr += phk[a] * __shfl(Tr[v], e0 + a * EW);
                }
            }
            const double from_w = __shfl(e, me >= 1 ? me - 1 : me);
            const double from_e = __shfl(w, me + 1 < 64 ? me + 1 : me);
            Ui[v] = w;
            Ei[v] = e;
            Wx[v] = gw ? tl : from_w;
            Ex[v] = ge ? tr : from_e;
        }
        edge_flux<CL, FX, 0, -1>(g, Ui, Wx, xc - 0.5 * g.dx, yk, hw);
        edge_flux<CL, FX, 0, 1>(g, Ei, Ex, xc + 0.5 * g.dx, yk, he);
        // west/east lifts of row r enter R[a][b] with the same weight
        // w_r phi_b(eta_r) as X[r][a]: X[r][a] = -(1/dx)(phi_a(-1) h_W + phi_a(1) h_E)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double hp = he[v] + hw[v], hm = he[v] - hw[v];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                X[v][a] = -((0.5 * B.pp[a]) * ((a & 1) ? hm : hp));
                Y[v][a] = 0.0;
            }
        }
        const double xk = xc + 0.5 * g.dx * xik;
        // south / north: own and exterior traces from the y collapses; both
        // fluxes are formed before either is stored over the collapses
        double hn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double si = 0.0, so = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                if constexpr (YL) {
                    si += phk[a] * S[LY::ti(0 * NV + v, a)];
                    so += phk[a] * S[LY::ti(2 * NV + v, a)];
                } else {
                    si += phk[a] * __shfl(Tm[v], e0 + a * EW);
                    so += phk[a] * __shfl(Tb[v], e0 + a * EW);
                }
            }
            Ui[v] = si;
            Uo[v] = so;
        }
        edge_flux<CL, FX, 1, -1>(g, Ui, Uo, xk, yc - 0.5 * g.dy, hs);
        if constexpr (!YL) {
#pragma unroll
            for (int v = 0; v < NV; ++v) S[LY::ti(0 * NV + v, k)] = hs[v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double si = 0.0, so = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                if constexpr (YL) {
                    si += phk[a] * S[LY::ti(1 * NV + v, a)];
                    so += phk[a] * S[LY::ti(3 * NV + v, a)];
                } else {
                    si += phk[a] * __shfl(Tp[v], e0 + a * EW);
                    so += phk[a] * __shfl(Tt[v], e0 + a * EW);
                }
            }
            Ui[v] = si;
            Uo[v] = so;
        }
        edge_flux<CL, FX, 1, 1>(g, Ui, Uo, xk, yc + 0.5 * g.dy, hn);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (YL) S[LY::ti(0 * NV + v, k)] = hs[v];
            S[LY::ti(1 * NV + v, k)] = hn[v];
        }
    }
    const double wk = pick<N>(B.wh, k) * g.dx * g.dy;  // torque: node mass factor of Gauss row k
    double tqs = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double W[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) s += B.phi[a][q] * Cc[v][a];
            W[v] = s;
        }
        const double x = xc + 0.5 * g.dx * B.xi[q];
        const double y = yk;
        const double inv = rcp64(W[0]);
        const double r2 = x * x + y * y;
        const double ir = (CL == CL_LOC || g.star) ? rsq64(r2) : 0.0;
        double p;
        if constexpr (CL == CL_ISO)
            p = g.cs2 * W[0];
        else if constexpr (CL == CL_LOC)
            p = cs2_loc(g, r2, ir) * W[0];
        else
            p = (g.gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) * inv);
        const double vx = W[1] * inv, vy = W[2] * inv;
        double gx = 0.0, gy = 0.0;
        if (g.star) {
            const double kk = r2 < g.rc2 ? g.rc3inv_h : g.gm_h * ir * ir * ir;
            gx = kk * x;
            gy = kk * y;
        }
        if (TQ || g.q > 0.0) {
            const double dx = x - xp, dy = y - yp;
            const double id = rsq64(dx * dx + dy * dy + g.eps2);
            const double id3 = id * id * id;
            const double kk = g.q_h * id3;
            gx += kk * dx;
            gy += kk * dy;
            if constexpr (TQ) tqs += torque_term(W[0], wk * B.wh[q], xp, yp, dx, dy, id3);
        }
        double fx[NV], fy[NV], sy[NV];
        fx[0] = W[1];
        fy[0] = W[2];
        sy[0] = 0.0;
        fx[1] = W[1] * vx + p;
        fy[1] = W[1] * vy;
        fx[2] = W[2] * vx;
        fy[2] = W[2] * vy + p;
        sy[1] = -W[0] * gx;
        sy[2] = -W[0] * gy;
        if constexpr (NV == 4) {
            fx[3] = (W[3] + p) * vx;
            fy[3] = (W[3] + p) * vy;
            sy[3] = -(W[1] * gx + W[2] * gy);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double fxx = fx[v], fyy = fy[v];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                // the density equation has no source term
                X[v][a] += v == 0 ? B.wdphi[a][q] * fxx : B.wdphi[a][q] * fxx + B.wphi[a][q] * sy[v];
                Y[v][a] += B.wphi[a][q] * fyy;
            }
        }
    }
    if constexpr (TQ) {
        const double t = wave_sum(active ? tqs : 0.0);
        if (lane == 0) tq_part[tile] = t;
    }
    __syncthreads();  // every lane has read C
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) S[LY::ci(v, k, a)] = X[v][a];
    __syncthreads();

    // ---- phase 3: k = mode row a
    double wrow[N];  // w_q phi_k(xi_q)
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double r = B.wphi[0][q];
#pragma unroll
        for (int m = 1; m < N; ++m) r = k == m ? B.wphi[m][q] : r;
        wrow[q] = r;
    }
    // R = a2 L(u) row by row: X and Y hold the x and y projections without
    // their 2/dx and 2/dy (the sources and the west/east lifts scaled by dx/2
    // instead), which go in with a2 here
    const double a2x = a2 * g.rdx2, a2y = a2 * g.rdy2, a2i = a2 * g.idy;
    double R[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double glb = 0.0, glt = 0.0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            glb += wrow[q] * S[LY::ti(0 * NV + v, q)];
            glt += wrow[q] * S[LY::ti(1 * NV + v, q)];
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < N; ++r) acc += B.wphi[b][r] * S[LY::ci(v, r, k)];
            R[v][b] = a2x * acc - a2i * (B.pm[b] * glb + B.pp[b] * glt);
        }
    }
    __syncthreads();  // every lane has read X
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) S[LY::ci(v, k, a)] = Y[v][a];
    __syncthreads();
    // the row's u^n, loaded before any store (out may alias u^n, so a load
    // after a store could not be moved ahead of it).  With three variables
    // the row's u stays in registers from phase 1 (reloading it this late
    // misses L2 for about a third more HBM reads per launch); with four the
    // registers are not there, and it is reloaded.
    constexpr bool keep_u = NV == 3;
    double Un[NV][N], U1[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int b = 0; b < N; ++b) U1[v][b] = keep_u ? Ua[v][b] : ld64(ru, vrow, (unsigned)(v * N + b) * RS);
    if (a0 != 0.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) Un[v][b] = ld64(run, vrow, (unsigned)(v * N + b) * RS);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int b = 0; b < N; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < N; ++r) acc += B.wdphi[b][r] * S[LY::ci(v, r, k)];
            R[v][b] += a2y * acc;
        }
    // the new row; with PP the positivity scaling of Sec. 2.4 on it before
    // the store (the same factors as the separate positivity pass on the
    // stored state, bit for bit)
    double O[NV][N];
    if (a0 != 0.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) O[v][b] = a0 * Un[v][b] + (a1 * U1[v][b] + R[v][b]);
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) O[v][b] = a1 * U1[v][b] + R[v][b];
    }
    if constexpr (PP != 0) {
        __syncthreads();  // every lane has read Y
        double th1, th2;
        pp_factors<N, NV>(g, S, k, O, g.pp_eps, th1, th2);
        if constexpr (PP == 1) {
            pp_scale_row<N, NV>(k, th1, th2, O);
        } else {
            const bool ok = __all(!active || (th1 >= 1.0 && th2 >= 1.0));
            if (lane == 0) pp_ok[tile] = ok ? 1 : 0;
        }
    }
    if (active) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) st64(rout, vrow, (unsigned)(v * N + b) * RS, O[v][b]);
    }
    if constexpr (MF) {
        static_assert(N == 4 && NV == 4, "the network takes 16 modes of 4 variables");
        MlpLane w;
        mlp_lane_from_pack(mlp_pack, lane, w);
        bf16x4 bfr[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // the element's mean is mode (0, 0), held by its lane k = 0 (lane e0)
            const double d = fabs(__shfl(O[v][0], e0)) + mlp_scale[v];
#pragma unroll
            for (int b = 0; b < 4; ++b) bfr[v][b] = active ? (short)f2bf((float)(O[v][b] / d)) : (short)0;
        }
        const float z = mlp_logit(w, bfr);
        if (active && k == 0) mlp_flags[(size_t)j * g.nx + i] = z > mlp_zthr ? 1 : 0;
    }
}

// ------------------------------------------------------------------ deviation form
// u = u_eq + du about the disc's rotational equilibrium u_eq (locally
// isothermal, stellar harmonic core inside r_core), u_eq being the projection
// of the analytic equilibrium.  The FP64 state du is converted to FP32 on load;
// contractions, fluxes and the lift run in FP32 on the deviation;
// L = L(u_eq) (FP64, computed once) + dL, and the stage combination is FP64.
// Every deviation term is linearised about u_eq's own polynomial: at the
// volume Gauss nodes the projection interpolates, so there the analytic
// equilibrium is u_eq's value; at the edge points u_eq's traces differ from
// the analytic profile by the projection error and are read from a table.
// Deviation fluxes are written without cancellation: with the equilibrium
// velocity v and w = dm - v drho,
//   d(m_a m_b / rho) = v_a v_b drho + v_a w_b + v_b w_a + w_a w_b / (rho + drho).
struct EqPoint {
    float rho, vx, vy, c2;
};

// the analytic equilibrium at a volume Gauss node
__device__ __forceinline__ EqPoint eq_at(const Geo& g, double xd, double yd) {
    const float x = (float)xd, y = (float)yd;
    const float r = sqrtf(x * x + y * y);
    const float rr = fmaxf(r, (float)g.r_core);
    EqPoint q;
    q.rho = (float)g.sigma0 * rsqrtf(rr);
    q.c2 = (float)g.h2gm / rr;
    const float om2 = r < (float)g.r_core ? (float)g.rc3inv : (float)(g.gm * (1.0 - 1.5 * g.h2gm / g.gm)) / (r * r * r);
    const float om = sqrtf(om2);
    q.vx = -om * y;
    q.vy = om * x;
    return q;
}

// u_eq's trace (rho, m_x, m_y) at an edge point, from the trace table, and the
// locally isothermal c_s^2 of that point
__device__ __forceinline__ EqPoint eq_trace(const float* e, float c2) {
    EqPoint q;
    q.rho = e[0];
    const float ir = 1.0f / e[0];
    q.vx = e[1] * ir;
    q.vy = e[2] * ir;
    q.c2 = c2;
    return q;
}

__device__ __forceinline__ float cs2_at(const Geo& g, double xd, double yd) {
    const float x = (float)xd, y = (float)yd;
    return (float)g.h2gm / fmaxf(sqrtf(x * x + y * y), (float)g.r_core);
}

// Trace table of u_eq: for every element, its own trace at the N points of its
// west, east, south and north edge (edges 0..3; points eta_k on the west/east
// edges, xi_k on the south/north edges), FP32, tiled like the state:
// entry (edge, v, k) of element (i, j) at eqtr_base + ((edge * 3 + v) * N + k) * EW.
template <int N>
__device__ __forceinline__ unsigned eqtr_base(const Geo& g, int i, int j) {
    constexpr int EW = tile_width(N);
    const int ti = i / EW;
    return (unsigned)(j * g.tiles_x + ti) * (unsigned)(4 * 3 * N * EW) + (unsigned)(i - ti * EW);
}

template <int AX>
__device__ __forceinline__ void dflux(const EqPoint& q, const float* d, float inv1, float* f) {
    const float wx = d[1] - q.vx * d[0], wy = d[2] - q.vy * d[0];
    const float dxy = q.vx * q.vy * d[0] + q.vx * wy + q.vy * wx + wx * wy * inv1;
    if constexpr (AX == 0) {
        f[0] = d[1];
        f[1] = q.vx * q.vx * d[0] + 2.0f * q.vx * wx + wx * wx * inv1 + q.c2 * d[0];
        f[2] = dxy;
    } else {
        f[0] = d[2];
        f[1] = dxy;
        f[2] = q.vy * q.vy * d[0] + 2.0f * q.vy * wy + wy * wy * inv1 + q.c2 * d[0];
    }
}

// normal velocity of the full state along SGN * e_AX
template <int AX, int SGN>
__device__ __forceinline__ float vnorm(const EqPoint& q, const float* d, float inv1) {
    const float v = AX == 0 ? q.vx + (d[1] - q.vx * d[0]) * inv1 : q.vy + (d[2] - q.vy * d[0]) * inv1;
    return SGN * v;
}

// Collapse of the exterior deviation across one edge for lane k (FP64 loaded,
// FP32 arithmetic): the neighbour's row k (ROW: modes (k, b), summed over b)
// or column k (modes (a, k), summed over a) with the basis values of its far
// side NB_SIDE, or, at a fixed box edge, the element's own initial row/column
// with the near side.  vnb / vown: byte offsets of mode (k, 0) resp. (0, k).
template <int N, bool ROW, int NB_SIDE>
__device__ __forceinline__ void ext_collapse_f(rsrc_t ru, rsrc_t ru0, unsigned vnb, unsigned vown, bool fixed,
                                               bool wave_fixed, float (&T)[3]) {
    constexpr BasisTab B = make_basis(N);
    constexpr int NN = N * N;
    constexpr unsigned RS = N * tile_width(N) * 8, CS = tile_width(N) * 8;
#pragma unroll
    for (int v = 0; v < 3; ++v) T[v] = 0.0f;
    if (!wave_fixed) {
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const unsigned so = ROW ? (unsigned)(v * N + m) * RS : (unsigned)(v * NN + m) * CS;
                T[v] += (float)(NB_SIDE > 0 ? B.pp[m] : B.pm[m]) * (float)ld64(ru, vnb, so);
            }
    } else {
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const unsigned so = ROW ? (unsigned)(v * N + m) * RS : (unsigned)(v * NN + m) * CS;
                const float un = (float)ld64(ru, vnb, so);
                const float u0v = (float)ld64(ru0, vown, so);
                T[v] += fixed ? (float)(NB_SIDE > 0 ? B.pm[m] : B.pp[m]) * u0v
                              : (float)(NB_SIDE > 0 ? B.pp[m] : B.pm[m]) * un;
            }
    }
}

// Rusanov flux of the deviation through an axis-aligned edge (outward normal
// SGN e_AX): F(ue_i + d_i, ue_o + d_o) - F(ue_i, ue_o) with the equilibrium
// traces ue_i, ue_o of the two sides (they differ by the projection error)
// and the locally isothermal sound speed shared by both sides.  The
// dissipation splits as -alpha (d_o - d_i) / 2 - (alpha - alpha_eq)(ue_o - ue_i) / 2.
template <int AX, int SGN>
__device__ __forceinline__ void rusanov_dev(const EqPoint& qi, const EqPoint& qo, const float* ei, const float* eo,
                                            const float* di, const float* dd, float* h) {
    const float ii = 1.0f / (qi.rho + di[0]), io = 1.0f / (qo.rho + dd[0]);
    float fi[3], fo[3];
    dflux<AX>(qi, di, ii, fi);
    dflux<AX>(qo, dd, io, fo);
    const float c = sqrtf(qi.c2);
    const float alpha = fmaxf(fabsf(vnorm<AX, SGN>(qi, di, ii)), fabsf(vnorm<AX, SGN>(qo, dd, io))) + c;
    const float alpha_eq = fmaxf(fabsf(AX == 0 ? qi.vx : qi.vy), fabsf(AX == 0 ? qo.vx : qo.vy)) + c;
    const float da = alpha - alpha_eq;
#pragma unroll
    for (int v = 0; v < 3; ++v)
        h[v] = 0.5f * SGN * (fi[v] + fo[v]) - 0.5f * alpha * (dd[v] - di[v]) - 0.5f * da * (eo[v] - ei[v]);
}

// Deviation-form stage with N lanes per element: the phases of k_stage_c in
// FP32 on the deviation (fluxes linearised about u_eq: the analytic profile at
// the volume nodes, u_eq's traces from the table at the edge points; stellar
// pull on the density deviation, planet on the full density), then
// out = a0 du^n + a1 du + a2 (L_eq + dL) in FP64.
template <int N>
__global__ void __launch_bounds__(64) k_stage_dev_c(const Geo g, int tiles_x, int tiles_total,
                                                    const double* __restrict__ du, const double* dun,
                                                    const double* __restrict__ du0, const double* __restrict__ leq,
                                                    const float* __restrict__ eqtr, double* out,
                                                    const StageCoeffs* __restrict__ scp, int rev) {
    constexpr int NV = 3;
    constexpr int NN = N * N;
    constexpr int EW = 64 / N;
    constexpr BasisTab B = make_basis(N);
    constexpr int P1 = NV * NN + 6 * NV * N;
    constexpr int P2 = 2 * NV * NN + 2 * NV * N;
    constexpr int SLOT = lds_slot_odd(P1 > P2 ? P1 : P2);
    __shared__ float lds[EW * SLOT];

    const int lane = threadIdx.x;
    // lane k * EW + s: index k of element slot s (rows contiguous in lane
    // order); lanes beyond N * EW shadow slot 0's element
    const bool own = lane < N * EW;
    const int k = own ? lane / EW : lane - N * EW;
    const int sl = own ? lane - k * EW : EW;
    const int tile = remap_tile(blockIdx.x, tiles_total, rev);
    const int j = tile / tiles_x;
    const int i0 = (tile - j * tiles_x) * EW;
    const bool active = sl < EW && i0 + sl < g.nx;
    const int i = active ? i0 + sl : i0;
    float* S = lds + (own ? sl : 0) * SLOT;

    const double a0 = scp->a0, a1 = scp->a1, a2 = scp->a2, xp = scp->xp, yp = scp->yp;
    const rsrc_t rdu = make_rsrc(du), rdu0 = make_rsrc(du0), rout = make_rsrc(out), rdun = make_rsrc(dun),
                 rleq = make_rsrc(leq), rtr = make_rsrc(eqtr);
    constexpr unsigned RS = N * EW * 8;  // byte stride of (v * N + b) in a row
    const unsigned eb = tiled_base<N, NV>(g, i, j);
    const unsigned vrow = (eb + k * EW) * 8u;  // mode (k, 0) of this element
    const double xc = g.x0 + (i + 0.5) * g.dx, yc = g.y0 + (j + 0.5) * g.dy;

    // ---- phase 1: k = mode row
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        float Ua[N];
#pragma unroll
        for (int b = 0; b < N; ++b) Ua[b] = (float)ld64(rdu, vrow, (unsigned)(v * N + b) * RS);
#pragma unroll
        for (int r = 0; r < N; ++r) {
            float c = 0.0f;
#pragma unroll
            for (int b = 0; b < N; ++b) c += Ua[b] * (float)B.phi[b][r];
            S[(v * N + k) * N + r] = c;
        }
        float tm = 0.0f, tp = 0.0f;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            tm += (float)B.pm[b] * Ua[b];
            tp += (float)B.pp[b] * Ua[b];
        }
        S[NV * NN + (0 * NV + v) * N + k] = tm;
        S[NV * NN + (1 * NV + v) * N + k] = tp;
    }
    int il = i - 1, ir = i + 1, jb = j - 1, jt = j + 1;
    const bool ol = il < 0, orr = ir >= g.nx, ob = jb < 0, ot = jt >= g.ny;
    il += ol ? g.nx : 0;
    ir -= orr ? g.nx : 0;
    jb += ob ? g.ny : 0;
    jt -= ot ? g.ny : 0;
    const bool fx = g.bc == 1, fl = fx && ol, fr = fx && orr, fb = fx && ob, ft = fx && ot;
    {
        const bool wfx = __any(fl || fr), wfy = __any(fb || ft);
        const unsigned vcol = (eb + k * N * EW) * 8u;
        float T[NV];
        ext_collapse_f<N, true, +1>(rdu, rdu0, (tiled_base<N, NV>(g, i, jb) + k * EW) * 8u, vrow, fb, wfy, T);
#pragma unroll
        for (int v = 0; v < NV; ++v) S[NV * NN + (2 * NV + v) * N + k] = T[v];
        ext_collapse_f<N, true, -1>(rdu, rdu0, (tiled_base<N, NV>(g, i, jt) + k * EW) * 8u, vrow, ft, wfy, T);
#pragma unroll
        for (int v = 0; v < NV; ++v) S[NV * NN + (3 * NV + v) * N + k] = T[v];
        ext_collapse_f<N, false, +1>(rdu, rdu0, (tiled_base<N, NV>(g, il, j) + k * N * EW) * 8u, vcol, fl, wfx, T);
#pragma unroll
        for (int v = 0; v < NV; ++v) S[NV * NN + (4 * NV + v) * N + k] = T[v];
        ext_collapse_f<N, false, -1>(rdu, rdu0, (tiled_base<N, NV>(g, ir, j) + k * N * EW) * 8u, vcol, fr, wfx, T);
#pragma unroll
        for (int v = 0; v < NV; ++v) S[NV * NN + (5 * NV + v) * N + k] = T[v];
    }
    __syncthreads();

    // ---- phase 2: k = Gauss row r
    const double xik = pick<N>(B.xi, k);
    float phk[N];
#pragma unroll
    for (int m = 0; m < N; ++m) phk[m] = (float)pick<N>(B.phi[m], k);
    const double yk = yc + 0.5 * g.dy * xik;
    float Cc[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) Cc[v][a] = S[(v * N + a) * N + k];
    float X[NV][N], Y[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) {
            X[v][a] = 0.0f;
            Y[v][a] = 0.0f;
        }
    const float rdx2 = (float)g.rdx2, rdy2 = (float)g.rdy2;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        float d[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            float s = 0.0f;
#pragma unroll
            for (int a = 0; a < N; ++a) s += (float)B.phi[a][q] * Cc[v][a];
            d[v] = s;
        }
        const double x = xc + 0.5 * g.dx * B.xi[q];
        const EqPoint qe = eq_at(g, x, yk);
        const float inv1 = 1.0f / (qe.rho + d[0]);
        float fx[NV], fy[NV], sy[NV];
        dflux<0>(qe, d, inv1, fx);
        dflux<1>(qe, d, inv1, fy);
        const float xf = (float)x, yf = (float)yk;
        const float r2 = xf * xf + yf * yf, rr = sqrtf(r2);
        const float ks = rr < (float)g.r_core ? (float)g.rc3inv : (float)g.gm / (r2 * rr);
        float gsx = -d[0] * ks * xf, gsy = -d[0] * ks * yf;
        if (g.q > 0.0) {
            const float dx = (float)(x - xp), dy = (float)(yk - yp);
            const float d2 = dx * dx + dy * dy + (float)g.eps2;
            const float kp = (float)g.q * rsqrtf(d2) / d2;
            const float rho = qe.rho + d[0];
            gsx -= rho * kp * dx;
            gsy -= rho * kp * dy;
        }
        sy[0] = 0.0f;
        sy[1] = gsx;
        sy[2] = gsy;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float fxx = rdx2 * fx[v], fyy = rdy2 * fy[v];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                // the density equation has no source term
                X[v][a] += v == 0 ? (float)B.wdphi[a][q] * fxx
                                  : (float)B.wdphi[a][q] * fxx + (float)B.wphi[a][q] * sy[v];
                Y[v][a] += (float)B.wphi[a][q] * fyy;
            }
        }
    }
    float hf[4][NV];
    {
        const float* Cl = S + NV * NN;
        float di[NV], dd[NV];
        // u_eq's traces at point k of the four edges, own and exterior (the
        // neighbour's trace on the shared edge; at a fixed box edge the
        // exterior state is u0 = u_eq + du0 of the element itself, so its
        // equilibrium part is the element's own trace there)
        float ew[2][NV], ee[2][NV], es[2][NV], en[2][NV];
        {
            const unsigned ob = eqtr_base<N>(g, i, j);
            const unsigned bw = fl ? ob : eqtr_base<N>(g, il, j), be = fr ? ob : eqtr_base<N>(g, ir, j);
            const unsigned bs = fb ? ob : eqtr_base<N>(g, i, jb), bn = ft ? ob : eqtr_base<N>(g, i, jt);
            auto at = [&](unsigned base, int edge, int v) {
                return ld32(rtr, (base + (unsigned)(((edge * 3 + v) * N + k) * EW)) * 4u, 0u);
            };
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                ew[0][v] = at(ob, 0, v);
                ew[1][v] = at(bw, fl ? 0 : 1, v);
                ee[0][v] = at(ob, 1, v);
                ee[1][v] = at(be, fr ? 1 : 0, v);
                es[0][v] = at(ob, 2, v);
                es[1][v] = at(bs, fb ? 2 : 3, v);
                en[0][v] = at(ob, 3, v);
                en[1][v] = at(bn, ft ? 3 : 2, v);
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            float si = 0.0f, so = 0.0f;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                si += (float)B.pm[a] * Cc[v][a];
                so += phk[a] * Cl[(4 * NV + v) * N + a];
            }
            di[v] = si;
            dd[v] = so;
        }
        {
            const float c2 = cs2_at(g, xc - 0.5 * g.dx, yk);
            rusanov_dev<0, -1>(eq_trace(ew[0], c2), eq_trace(ew[1], c2), ew[0], ew[1], di, dd, hf[0]);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            float si = 0.0f, so = 0.0f;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                si += (float)B.pp[a] * Cc[v][a];
                so += phk[a] * Cl[(5 * NV + v) * N + a];
            }
            di[v] = si;
            dd[v] = so;
        }
        {
            const float c2 = cs2_at(g, xc + 0.5 * g.dx, yk);
            rusanov_dev<0, 1>(eq_trace(ee[0], c2), eq_trace(ee[1], c2), ee[0], ee[1], di, dd, hf[1]);
        }
        // west/east lifts folded into X (same weight w_r phi_b(eta_r) in R)
        const float idx = (float)g.idx;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float hp = idx * (hf[1][v] + hf[0][v]), hm = idx * (hf[1][v] - hf[0][v]);
#pragma unroll
            for (int a = 0; a < N; ++a) X[v][a] -= (float)B.pp[a] * ((a & 1) ? hm : hp);
        }
        const double xk = xc + 0.5 * g.dx * xik;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            float si = 0.0f, so = 0.0f;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                si += phk[a] * Cl[(0 * NV + v) * N + a];
                so += phk[a] * Cl[(2 * NV + v) * N + a];
            }
            di[v] = si;
            dd[v] = so;
        }
        {
            const float c2 = cs2_at(g, xk, yc - 0.5 * g.dy);
            rusanov_dev<1, -1>(eq_trace(es[0], c2), eq_trace(es[1], c2), es[0], es[1], di, dd, hf[2]);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            float si = 0.0f, so = 0.0f;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                si += phk[a] * Cl[(1 * NV + v) * N + a];
                so += phk[a] * Cl[(3 * NV + v) * N + a];
            }
            di[v] = si;
            dd[v] = so;
        }
        {
            const float c2 = cs2_at(g, xk, yc + 0.5 * g.dy);
            rusanov_dev<1, 1>(eq_trace(en[0], c2), eq_trace(en[1], c2), en[0], en[1], di, dd, hf[3]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) {
            S[((0 * NV + v) * N + k) * N + a] = X[v][a];
            S[((1 * NV + v) * N + k) * N + a] = Y[v][a];
        }
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int v = 0; v < NV; ++v) S[2 * NV * NN + (f * NV + v) * N + k] = hf[2 + f][v];
    __syncthreads();

    // ---- phase 3: k = mode row a
    float wrow[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double r = B.wphi[0][q];
#pragma unroll
        for (int m = 1; m < N; ++m) r = k == m ? B.wphi[m][q] : r;
        wrow[q] = (float)r;
    }
    const float idy = (float)g.idy;
    const float* H = S + 2 * NV * NN;
    // L_eq, du and du^n of the row, issued before any store (out may alias du^n)
    double Le[NV][N];
    double U1[NV][N], Un[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int b = 0; b < N; ++b) {
            Le[v][b] = ld64(rleq, vrow, (unsigned)(v * N + b) * RS);
            U1[v][b] = ld64(rdu, vrow, (unsigned)(v * N + b) * RS);
        }
    if (a0 != 0.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) Un[v][b] = ld64(rdun, vrow, (unsigned)(v * N + b) * RS);
    }
    float R[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        float glb = 0.0f, glt = 0.0f;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            glb += wrow[q] * H[(0 * NV + v) * N + q];
            glt += wrow[q] * H[(1 * NV + v) * N + q];
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            float acc = 0.0f;
#pragma unroll
            for (int r = 0; r < N; ++r)
                acc += (float)B.wphi[b][r] * S[((0 * NV + v) * N + r) * N + k] +
                       (float)B.wdphi[b][r] * S[((1 * NV + v) * N + r) * N + k];
            acc -= idy * ((float)B.pm[b] * glb + (float)B.pp[b] * glt);
            R[v][b] = acc;
        }
    }
    if (active) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const unsigned po = (unsigned)(v * N + b) * RS;
                const double L = Le[v][b] + (double)R[v][b];
                const double base = a1 * U1[v][b] + a2 * L;
                st64(rout, vrow, po, a0 != 0.0 ? a0 * Un[v][b] + base : base);
            }
    }
}

// out = a + sign * b, elementwise over a state array (out may alias b)
__global__ void k_add_state(const double* a, const double* b, double* out, double sign, long long n) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k < n) out[k] = a[k] + sign * b[k];
}

// trace table of the projected equilibrium (layout at eqtr_base): thread per
// element, the polynomial of its modes at the N points of each edge
template <int N>
__global__ void __launch_bounds__(64) k_eq_traces(const Geo g, const double* __restrict__ eq, float* __restrict__ eqtr) {
    constexpr BasisTab T = make_basis(N);
    constexpr int EW = tile_width(N);
    const long long e = (long long)blockIdx.x * 64 + threadIdx.x;
    if (e >= g.E) return;
    const int i = (int)(e % g.nx), j = (int)(e / g.nx);
    const unsigned base = tiled_base<N, 3>(g, i, j), tb = eqtr_base<N>(g, i, j);
    for (int v = 0; v < 3; ++v)
        for (int k = 0; k < N; ++k) {
            double w = 0.0, ea = 0.0, so = 0.0, no = 0.0;
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) {
                    const double c = eq[base + mode_off<N>(v, a, b)];
                    w += c * T.pm[a] * T.phi[b][k];
                    ea += c * T.pp[a] * T.phi[b][k];
                    so += c * T.phi[a][k] * T.pm[b];
                    no += c * T.phi[a][k] * T.pp[b];
                }
            eqtr[tb + ((0 * 3 + v) * N + k) * EW] = (float)w;
            eqtr[tb + ((1 * 3 + v) * N + k) * EW] = (float)ea;
            eqtr[tb + ((2 * 3 + v) * N + k) * EW] = (float)so;
            eqtr[tb + ((3 * 3 + v) * N + k) * EW] = (float)no;
        }
}

// ------------------------------------------------------------------ init
template <int N, int NV>
__global__ void __launch_bounds__(64) k_project(const Geo g, const double* __restrict__ prim,
                                                double* __restrict__ u) {
    constexpr int NN = N * N;
    constexpr BasisTab T = make_basis(N);
    const long long e = (long long)blockIdx.x * 64 + threadIdx.x;
    if (e >= g.E) return;
    const long long E = g.E;
    const unsigned base = tiled_base<N, NV>(g, (int)(e % g.nx), (int)(e / g.nx));
    double C[NV][NN];
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        const double rho = prim[(0 * E + e) * NN + k];
        const double vx = prim[(1 * E + e) * NN + k];
        const double vy = prim[(2 * E + e) * NN + k];
        C[0][k] = rho;
        C[1][k] = rho * vx;
        C[2][k] = rho * vy;
        if constexpr (NV == 4) {
            const double p = prim[(3 * E + e) * NN + k];
            C[3][k] = p / (g.gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int b = 0; b < N; ++b) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < N; ++q)
#pragma unroll
                    for (int r = 0; r < N; ++r)
                        s += C[v][q * N + r] * (T.wh[q] * T.wh[r] * T.phi[a][q] * T.phi[b][r]);
                u[base + mode_off<N>(v, a, b)] = s;
            }
}

// means of every variable of element e into out[v * E + e]
template <int N, int NV>
__global__ void __launch_bounds__(256) k_means(const Geo g, const double* __restrict__ u, double* __restrict__ out) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.E) return;
    const unsigned base = tiled_base<N, NV>(g, (int)(e % g.nx), (int)(e / g.nx));
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * g.E + e] = u[base + mode_off<N>(v, 0, 0)];
}

// ------------------------------------------------------------------ small kernels
__device__ __forceinline__ void planet_at(const Geo& g, double t, double& xp, double& yp) {
    double sn, cs;
    sincos(g.omp * t + g.phi0, &sn, &cs);
    xp = g.rp * cs;
    yp = g.rp * sn;
}

__global__ void k_set_coeffs(StageCoeffs* sc, const Geo g, double t, double a0, double a1, double a2) {
    StageCoeffs c;
    c.t = t;
    planet_at(g, t, c.xp, c.yp);
    c.a0 = a0;
    c.a1 = a1;
    c.a2 = a2;
    c.dt = 0.0;
    c.pad = 0.0;
    *sc = c;
}

// Minimum of the per-block CFL steps and OR of the per-block flags, over one
// block of 256 threads; the result is valid in thread 0.  The flags are
// merged into sb->flags (read and cleared by the host).
__device__ double reduce_dt_partials(const double* __restrict__ dt_part, const unsigned int* __restrict__ bad_part,
                                     int nblk, StepBlock* sb) {
    __shared__ double sm[256];
    __shared__ unsigned int sf[256];
    double m = INFINITY;
    unsigned int f = 0;
    for (int k = threadIdx.x; k < nblk; k += 256) {
        m = fmin(m, dt_part[k]);
        f |= bad_part[k];
    }
    sm[threadIdx.x] = m;
    sf[threadIdx.x] = f;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + w]);
            sf[threadIdx.x] |= sf[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && sf[0]) sb->flags |= 1u;
    return sm[0];
}

// Shu-Osher convex forms: SSP(3,3) (nst = 3, c = (0, 1, 1/2)) and SSP(2,2)
// as Heun (nst = 2, c = (0, 1)): u^(i+1) = a0 u^n + a1 (u^(i) + dt L(u^(i))).
// One block of 256 threads.
__global__ void __launch_bounds__(256) k_step_begin(const Geo g, StepBlock* sb, const double* __restrict__ dt_part,
                                                    const unsigned int* __restrict__ bad_part, int nblk,
                                                    double* t_dev, double dt_fixed, double* dt_used, int nst) {
    const double dtmin = reduce_dt_partials(dt_part, bad_part, nblk, sb);
    const double t = *t_dev;
    __syncthreads();  // every thread has read t^n before thread 0 advances it
    const double dt = dt_fixed > 0.0 ? dt_fixed : dtmin;
    const int s = threadIdx.x;  // one thread per stage (the planet positions in parallel)
    if (s < nst) {
        const bool two = nst == 2;
        const double cst[3] = {0.0, 1.0, 0.5};
        const double a0[3] = {0.0, two ? 0.5 : 0.75, 1.0 / 3.0};
        const double a1[3] = {1.0, two ? 0.5 : 0.25, 2.0 / 3.0};
        const double a2[3] = {1.0, two ? 0.5 : 0.25, 2.0 / 3.0};
        StageCoeffs c;
        c.t = t + cst[s] * dt;
        planet_at(g, c.t, c.xp, c.yp);
        c.a0 = a0[s];
        c.a1 = a1[s];
        c.a2 = a2[s] * dt;
        c.dt = dt;
        c.pad = 0.0;
        sb->st[s] = c;
    }
    if (s == 0) {
        *t_dev = t + dt;
        if (dt_used) *dt_used = dt;
    }
}

// Butcher-form step: stage times and planet positions, k_i = L(y_i)
// coefficients, and the dt-scaled combination rows, from the device dt
__global__ void __launch_bounds__(256) k_step_begin_table(const Geo g, StepBlock* sb, const RKTable tab,
                                                          const double* __restrict__ dt_part,
                                                          const unsigned int* __restrict__ bad_part, int nblk,
                                                          double* t_dev, double dt_fixed, double* dt_used) {
    const double dtmin = reduce_dt_partials(dt_part, bad_part, nblk, sb);
    if (threadIdx.x != 0) return;
    const double t = *t_dev;
    const double dt = dt_fixed > 0.0 ? dt_fixed : dtmin;
    for (int i = 0; i < tab.s; ++i) {
        StageCoeffs c;
        c.t = t + tab.c[i] * dt;
        planet_at(g, c.t, c.xp, c.yp);
        c.a0 = 0.0;
        c.a1 = 0.0;
        c.a2 = 1.0;
        c.dt = dt;
        c.pad = 0.0;
        sb->st[i] = c;
        for (int j = 0; j < kMaxStages; ++j) {
            sb->comb[i][j] = i == 0 ? (j < tab.s ? dt * tab.b[j] : 0.0)
                                    : (j < i ? dt * tab.A[i * kMaxStages + j] : 0.0);
        }
    }
    *t_dev = t + dt;
    if (dt_used) *dt_used = dt;
}

struct KPtrs {
    const double* k[kMaxStages];
};

// out = base + sum_j coef[j] k_j, element-wise (out may alias base)
__global__ void __launch_bounds__(256) k_rk_combine(const double* base, const KPtrs kp, int nk,
                                                    const double* __restrict__ coef, double* out, long long n) {
    const long long x = (long long)blockIdx.x * 256 + threadIdx.x;
    if (x >= n) return;
    double acc = 0.0;
    for (int j = 0; j < nk; ++j) acc = fma(coef[j], kp.k[j][x], acc);
    out[x] = base[x] + acc;
}

// CFL step of Sec. 2.3 per element from its means; the block minimum and
// the block's flag go to per-block slots, reduced by the step-begin kernel
// (no atomics: a fixed reduction order and no cross-kernel atomic traffic).
template <int CL>
__global__ void __launch_bounds__(256) k_dt(const Geo g, int nn, const double* __restrict__ u,
                                            const double* __restrict__ eq, double* __restrict__ dt_part,
                                            unsigned int* __restrict__ bad_part) {
    __shared__ double red[4];
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    double dte = INFINITY;
    bool bad = false;
    if (e < g.E) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        // tiled layout with a run-time tile width: mean of variable v at
        // base + v * nn * ew
        constexpr int NV = CL == CL_ADI ? 4 : 3;
        const int ti = i / g.ew;
        const unsigned vs = (unsigned)(nn * g.ew);
        const unsigned base = (unsigned)(j * g.tiles_x + ti) * (unsigned)NV * vs + (unsigned)(i - ti * g.ew);
        double U[4];
        U[0] = u[base];
        U[1] = u[base + vs];
        U[2] = u[base + 2 * vs];
        U[3] = CL == CL_ADI ? u[base + 3 * vs] : 0.0;
        if (eq) {  // deviation form: means of u_eq + du
            U[0] += eq[base];
            U[1] += eq[base + vs];
            U[2] += eq[base + 2 * vs];
        }
        const double xc = g.x0 + (i + 0.5) * g.dx, yc = g.y0 + (j + 0.5) * g.dy;
        double p, c;
        pressure<CL>(g, U, 1.0 / U[0], xc, yc, p, c);
        const double sx = (fabs(U[1] / U[0]) + c) / g.dx;
        const double sy = (fabs(U[2] / U[0]) + c) / g.dy;
        dte = g.cfl_fac / (sx + sy);
        bad = !(U[0] > 0.0) || !(dte > 0.0) || !isfinite(dte);
        if (bad) dte = INFINITY;
    }
    for (int off = 32; off > 0; off >>= 1) dte = fmin(dte, __shfl_xor(dte, off));
    const int anybad = __syncthreads_or(bad ? 1 : 0);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = dte;
    __syncthreads();
    if (threadIdx.x == 0) {
        dt_part[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
        bad_part[blockIdx.x] = anybad ? 1u : 0u;
    }
}

// ------------------------------------------------------------------ damping
// ramp R(r) of the wave-killing zones and the zone's damping period T_d
__device__ __forceinline__ double ramp(const Geo& g, double r, double& td) {
    if (r < g.rd_in) {
        const double s = (r - g.rd_in) * g.irw_in;
        td = g.td_in;
        return s > 1.0 ? 1.0 : s * s;
    }
    if (r > g.rd_out) {
        const double s = (r - g.rd_out) * g.irw_out;
        td = g.td_out;
        return s > 1.0 ? 1.0 : s * s;
    }
    td = g.td_in;
    return 0.0;
}

// Damping targets: rho0, v0x, v0y (and T0 with four variables) of u0 at the
// Gauss nodes of every listed tile, q0[list index][v][q][r][slot], computed
// once at set-up by N lanes per element (lane k: mode row k of u0, then
// Gauss row k), with the arithmetic the damping used when it contracted u0
// at every step.
template <int N, int CL>
__global__ void __launch_bounds__(64) k_damp_prep(const Geo g, const double* __restrict__ u0,
                                                  const int* __restrict__ list, double* __restrict__ q0) {
    constexpr BasisTab B = make_basis(N);
    constexpr int NV = NVar<CL>::value;
    constexpr int EW = 64 / N;
    constexpr int SLOT = lds_slot_odd(NV * N * N);
    __shared__ double lds[EW * SLOT];
    constexpr unsigned RS = N * EW * 8;
    const int lane = threadIdx.x;
    // lane k * EW + s: index k of element slot s (rows contiguous in lane
    // order); lanes beyond N * EW shadow slot 0's element
    const bool own = lane < N * EW;
    const int k = own ? lane / EW : lane - N * EW;
    const int sl = own ? lane - k * EW : EW;
    const int tile = list[blockIdx.x];
    const int j = tile / g.tiles_x;
    const int i0 = (tile - j * g.tiles_x) * EW;
    const int i = (sl < EW && i0 + sl < g.nx) ? i0 + sl : i0;
    double* S = lds + (own ? sl : 0) * SLOT;
    const rsrc_t ru0 = make_rsrc(u0);
    const unsigned vrow = (tiled_base<N, NV>(g, i, j) + k * EW) * 8u;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double A0[N];
#pragma unroll
        for (int b = 0; b < N; ++b) A0[b] = ld64(ru0, vrow, (unsigned)(v * N + b) * RS);
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double c0 = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) c0 += A0[b] * B.phi[b][r];
            S[(v * N + k) * N + r] = c0;
        }
    }
    __syncthreads();
    double C0[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) C0[v][a] = S[(v * N + a) * N + k];
    const unsigned qs = (unsigned)(N * EW);  // stride of (v, q) in q0
    double* qb = q0 + (size_t)blockIdx.x * NV * N * qs + k * EW + (own ? sl : 0);
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double W0[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s0 = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) s0 += B.phi[a][q] * C0[v][a];
            W0[v] = s0;
        }
        const double rho0 = W0[0], ir0 = rcp64(rho0), vx0 = W0[1] * ir0, vy0 = W0[2] * ir0;
        double P0[NV];
        P0[0] = rho0;
        P0[1] = vx0;
        P0[2] = vy0;
        if constexpr (NV == 4) {
            const double gm1 = g.gamma - 1.0;
            P0[3] = gm1 * (W0[3] - 0.5 * rho0 * (vx0 * vx0 + vy0 * vy0)) * ir0;
        }
        if (own) {
#pragma unroll
            for (int v = 0; v < NV; ++v) qb[(v * N + q) * qs] = P0[v];
        }
    }
}

// Damping with N lanes per element (same split as k_stage_c): lane k first
// holds mode row k of u and contracts it in y, then Gauss row k (node values,
// nodal increments against the targets of k_damp_prep, x projection), then
// mode row k again (y projection and the update).  One listed tile (EW = 64 /
// N elements) per wave; elements of the tile outside the damping zones get
// zero increments.
template <int N, int CL>
__global__ void __launch_bounds__(64) k_damp_c(const Geo g, double* u, const double* __restrict__ q0,
                                               const double* __restrict__ eq, const int* __restrict__ list, int nlist,
                                               const StageCoeffs* __restrict__ scp, int rev) {
    constexpr BasisTab B = make_basis(N);
    constexpr int NV = NVar<CL>::value;
    constexpr int NN = N * N;
    constexpr int EW = 64 / N;
    constexpr int SLOT = lds_slot_odd(NV * NN);
    __shared__ double lds[EW * SLOT];
    constexpr unsigned RS = N * EW * 8;  // byte stride of (v * N + b) in a row
    const int lane = threadIdx.x;
    // lane k * EW + s: index k of element slot s (rows contiguous in lane
    // order); lanes beyond N * EW shadow slot 0's element
    const bool own = lane < N * EW;
    const int k = own ? lane / EW : lane - N * EW;
    const int sl = own ? lane - k * EW : EW;
    // rev: the list from its end (the list is ordered by the tile's place in
    // its XCD band; the damping starts where the last stage ended)
    const int li = rev ? nlist - 1 - (int)blockIdx.x : (int)blockIdx.x;
    const int tile = list[li];
    const int j = tile / g.tiles_x;
    const int i0 = (tile - j * g.tiles_x) * EW;
    const bool active = sl < EW && i0 + sl < g.nx;
    const int i = active ? i0 + sl : i0;  // idle lanes shadow a valid element and store nothing
    double* S = lds + (own ? sl : 0) * SLOT;
    const double dt = scp->dt;
    const double xc = g.x0 + (i + 0.5) * g.dx, yc = g.y0 + (j + 0.5) * g.dy;
    const rsrc_t ru = make_rsrc(u), req = make_rsrc(eq ? eq : u);
    const unsigned vrow = (tiled_base<N, NV>(g, i, j) + k * EW) * 8u;  // mode (k, 0)

    // the targets of Gauss row k (loaded first, used in the second phase)
    const unsigned qs = (unsigned)(N * EW);
    const double* qb = q0 + (size_t)li * NV * N * qs + k * EW + (own ? sl : 0);
    double Tg[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < N; ++q) Tg[v][q] = qb[(v * N + q) * qs];

    // mode row k: y contraction of u (full state)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double A[N];
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const unsigned so = (unsigned)(v * N + b) * RS;
            const double ud = ld64(ru, vrow, so);
            A[b] = eq ? ld64(req, vrow, so) + ud : ud;
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double c = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) c += A[b] * B.phi[b][r];
            S[(v * N + k) * N + r] = c;
        }
    }
    __syncthreads();

    // Gauss row k: nodal increments, projected in x
    const double yk = yc + 0.5 * g.dy * pick<N>(B.xi, k);
    double Cc[NV][N], P[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) {
            Cc[v][a] = S[(v * N + a) * N + k];
            P[v][a] = 0.0;
        }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double W[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) s += B.phi[a][q] * Cc[v][a];
            W[v] = s;
        }
        const double x = xc + 0.5 * g.dx * B.xi[q];
        double td;
        const double R = ramp(g, sqrt(x * x + yk * yk), td);
        double D[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) D[v] = 0.0;
        if (R > 0.0) {
            const double w = dt * R * rcp64(td + dt * R);
            const double rho = W[0], ir = rcp64(rho), vx = W[1] * ir, vy = W[2] * ir;
            const double rho0 = Tg[0][q], vx0 = Tg[1][q], vy0 = Tg[2][q];
            const double drho = w * (rho0 - rho);
            const double dvx = w * (vx0 - vx), dvy = w * (vy0 - vy);
            const double vx1 = vx + dvx, vy1 = vy + dvy;
            D[0] = drho;
            D[1] = rho * dvx + drho * vx1;
            D[2] = rho * dvy + drho * vy1;
            if constexpr (NV == 4) {
                const double gm1 = g.gamma - 1.0;
                const double T1 = gm1 * (W[3] - 0.5 * rho * (vx * vx + vy * vy)) * ir;
                const double dT = w * (Tg[3][q] - T1);  // Tg[3]: the target temperature
                const double dp = rho * dT + drho * (T1 + dT);
                const double dke = 0.5 * (drho * (vx1 * vx1 + vy1 * vy1) + rho * (dvx * (vx1 + vx) + dvy * (vy1 + vy)));
                D[3] = dp / gm1 + dke;
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int a = 0; a < N; ++a) P[v][a] += B.wphi[a][q] * D[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < N; ++a) S[(v * N + k) * N + a] = P[v][a];
    __syncthreads();

    // mode row k: y projection and update; the row of u comes back from L2
    // (fewer live registers across the phases), all loads before the stores
    if (active) {
        double Ud[NV][N];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) Ud[v][b] = ld64(ru, vrow, (unsigned)(v * N + b) * RS);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) {
                double s = 0.0;
#pragma unroll
                for (int r = 0; r < N; ++r) s += B.wphi[b][r] * S[(v * N + r) * N + k];
                st64(ru, vrow, (unsigned)(v * N + b) * RS, Ud[v][b] + s);
            }
    }
}

// ------------------------------------------------------------------ torque

// deterministic block sum: fixed xor-butterfly inside each wavefront, then the
// wavefront sums in index order by thread 0 (its return value; other threads
// get 0)
template <int WAVES>
__device__ __forceinline__ double block_sum(double s, double* red) {
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < WAVES; ++w) r += red[w];
    return r;
}

// N lanes per element, one tile (EW = 64 / N elements of a row) per
// wavefront, four tiles per block, with the arithmetic of the stage kernel's
// phases 1 and 2: lane k contracts the density row k in y (LDS), then takes
// the nodes (xi_q, eta_k), q < N; one partial per tile (the wavefront's sum by
// a fixed butterfly), so the sum is bitwise reproducible and equal to the one
// the first stage kernel forms on the same state.
template <int N>
__global__ void __launch_bounds__(64 * kTorqueWaves) k_torque(const Geo g, double t, const double* t_dev,
                                                              const double* __restrict__ u,
                                                              const double* __restrict__ eq,
                                                              double* __restrict__ partials) {
    constexpr BasisTab B = make_basis(N);
    constexpr int EW = 64 / N;
    constexpr int TS = (N * N) | 1;  // slot stride: odd, the slots of one k on distinct banks
    __shared__ double lds[kTorqueWaves][EW * TS];
    __shared__ double pxy[2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // lane k * EW + s: index k of element slot s (rows contiguous in lane
    // order); lanes beyond N * EW shadow slot 0's element and add nothing
    const bool own = lane < N * EW;
    const int k = own ? lane / EW : lane - N * EW;
    const int sl = own ? lane - k * EW : EW;
    const int tile = blockIdx.x * kTorqueWaves + wv;
    const bool live = tile < g.tiles_x * g.ny;  // the last block may hold fewer tiles
    const int j = live ? tile / g.tiles_x : 0;
    const int i0 = live ? (tile - j * g.tiles_x) * EW : 0;
    const bool active = live && sl < EW && i0 + sl < g.nx;
    const int i = active ? i0 + sl : i0;
    double* S = lds[wv] + (own ? sl : 0) * TS;
    if (threadIdx.x == 0) {
        const double tt = t_dev ? *t_dev : t;
        planet_at(g, tt, pxy[0], pxy[1]);
    }
    // density row k (the variable count only sets the tile stride)
    const unsigned base = g.closure == 2 ? tiled_base<N, 4>(g, i, j) : tiled_base<N, 3>(g, i, j);
    double row[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        const unsigned idx = base + mode_off<N>(0, k, b);
        row[b] = eq ? eq[idx] + u[idx] : u[idx];
    }
    if (own) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double c = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) c += row[b] * B.phi[b][r];
            S[k * N + r] = c;
        }
    }
    __syncthreads();
    const double xp = pxy[0], yp = pxy[1];
    double Cc[N];
#pragma unroll
    for (int a = 0; a < N; ++a) Cc[a] = S[a * N + k];
    const double xc = g.x0 + (i + 0.5) * g.dx, yc = g.y0 + (j + 0.5) * g.dy;
    const double y = yc + 0.5 * g.dy * pick<N>(B.xi, k);
    const double wk = pick<N>(B.wh, k) * g.dx * g.dy;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double rho = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) rho += B.phi[a][q] * Cc[a];
        const double x = xc + 0.5 * g.dx * B.xi[q];
        const double dx = x - xp, dy = y - yp;
        const double id = rsq64(dx * dx + dy * dy + g.eps2);
        const double id3 = id * id * id;
        s += torque_term(rho, wk * B.wh[q], xp, yp, dx, dy, id3);
    }
    s = wave_sum(active ? s : 0.0);
    if (lane == 0 && live) partials[tile] = s;
}

// one block: thread p adds the partials p, p + 1024, ... in order (eight
// loads issued before their adds), then the block sum in a fixed order
__global__ void __launch_bounds__(kTorqueFinal) k_torque_final(const double* __restrict__ partials, int nb,
                                                               double* __restrict__ out) {
    __shared__ double red[kTorqueFinal / 64];
    double s = 0.0;
    int k = threadIdx.x;
    for (; k + 7 * kTorqueFinal < nb; k += 8 * kTorqueFinal) {
        double v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = partials[k + m * kTorqueFinal];
#pragma unroll
        for (int m = 0; m < 8; ++m) s += v[m];
    }
    for (; k < nb; k += kTorqueFinal) s += partials[k];
    const double b = block_sum<kTorqueFinal / 64>(s, red);
    if (threadIdx.x == 0) *out = b;
}

// ------------------------------------------------------------------ launchers
#define DG_DISPATCH_N(n, BODY)               \
    switch (n) {                             \
        case 2: { constexpr int NT = 2; BODY; } break; \
        case 3: { constexpr int NT = 3; BODY; } break; \
        case 4: { constexpr int NT = 4; BODY; } break; \
        case 5: { constexpr int NT = 5; BODY; } break; \
        default: return hipErrorInvalidValue;  \
    }

#define DG_DISPATCH_CL(cl, BODY)             \
    switch (cl) {                            \
        case CL_ISO: { constexpr int CT = CL_ISO; BODY; } break; \
        case CL_LOC: { constexpr int CT = CL_LOC; BODY; } break; \
        case CL_ADI: { constexpr int CT = CL_ADI; BODY; } break; \
        default: return hipErrorInvalidValue;  \
    }

hipError_t launch_project(int n, int nvar, const Geo& g, const double* prim, double* u, hipStream_t s) {
    const int blocks = (int)((g.E + 63) / 64);
    if (nvar == 4) {
        DG_DISPATCH_N(n, hipLaunchKernelGGL((k_project<NT, 4>), dim3(blocks), dim3(64), 0, s, g, prim, u));
    } else {
        DG_DISPATCH_N(n, hipLaunchKernelGGL((k_project<NT, 3>), dim3(blocks), dim3(64), 0, s, g, prim, u));
    }
    return hipGetLastError();
}

hipError_t launch_stage(int n, const Geo& g, const double* u, const double* un, const double* u0, double* out,
                        const StageCoeffs* sc, bool pp, double* tq_part, hipStream_t s, const MlpFlags* mf,
                        unsigned char* pp_ok, bool rev, const double* tq_sum, double* tq_out) {
    // arrays that a launch does not read still get a valid base (buffer
    // resources are never built on a null pointer)
    if (!un) un = u;
    if (!u0) u0 = u;
    // with the positivity scaling fused the torque terms take the order-5
    // adiabatic kernel past 256 registers (one wave per SIMD): not offered
    if (pp && tq_part) return hipErrorInvalidValue;
    // the torque partials of the first stage added up in a later one
    if ((tq_out != nullptr) != (tq_sum != nullptr) || (tq_out && tq_part)) return hipErrorInvalidValue;
    double* tq_arg = tq_part ? tq_part : const_cast<double*>(tq_sum);
    const int lead = tq_out ? 8 : 0;
    if (mf && (pp || n != 4 || g.closure != CL_ADI || !mf->pack || !mf->scale || !mf->flags))
        return hipErrorInvalidValue;
    if (pp_ok && (pp || n != 4 || g.closure != CL_ADI)) return hipErrorInvalidValue;
    const void* mpack = mf ? mf->pack : nullptr;
    const double* mscale = mf ? mf->scale : nullptr;
    unsigned char* mflags = mf ? mf->flags : nullptr;
    const float mzthr = mf ? mf->zthr : 0.f;
#define DG_STAGE(PPV, TQV, FXV, MFV)                                                                             \
    hipLaunchKernelGGL((k_stage_c<NT, CT, PPV, TQV, FXV, MFV>), dim3(tt + lead), dim3(64), 0, s, g, tx, tt, u, un, \
                       u0, out, sc, tq_arg, mpack, mscale, mflags, mzthr, pp_ok, rev ? 1 : 0, tq_out)
#define DG_STAGE_MF(TQV, FXV)                                      \
    if constexpr (NT == 4 && CT == CL_ADI) {                       \
        if (pp_ok) {                                               \
            if (mf)                                                \
                DG_STAGE(2, TQV, FXV, true);                       \
            else                                                   \
                DG_STAGE(2, TQV, FXV, false);                      \
        } else if (mf) {                                           \
            DG_STAGE(0, TQV, FXV, true);                           \
        } else {                                                   \
            DG_STAGE(0, TQV, FXV, false);                          \
        }                                                          \
    } else {                                                       \
        DG_STAGE(0, TQV, FXV, false);                              \
    }
#define DG_STAGE_FX(FXV)                       \
    if (pp) {                                  \
        DG_STAGE(1, false, FXV, false);        \
    } else if (tq_part) {                      \
        DG_STAGE_MF(true, FXV)                 \
    } else {                                   \
        DG_STAGE_MF(false, FXV)                \
    }
    DG_DISPATCH_CL(g.closure, DG_DISPATCH_N(n, {
        constexpr int EW = 64 / NT;
        const int tx = (g.nx + EW - 1) / EW;
        const int tt = tx * g.ny;
        if constexpr (CT == CL_ADI) {
            if (g.flux == 1) {
                DG_STAGE_FX(1);
            } else {
                DG_STAGE_FX(0);
            }
        } else {
            DG_STAGE_FX(0);
        }
    }));
#undef DG_STAGE_FX
#undef DG_STAGE_MF
#undef DG_STAGE
    return hipGetLastError();
}

hipError_t launch_set_coeffs(StageCoeffs* sc, const Geo& g, double t, double a0, double a1, double a2,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_set_coeffs, dim3(1), dim3(1), 0, s, sc, g, t, a0, a1, a2);
    return hipGetLastError();
}

int dt_blocks(const Geo& g) { return (int)((g.E + 255) / 256); }

hipError_t launch_means(int n, int nvar, const Geo& g, const double* u, double* out, hipStream_t s) {
    const int blocks = (int)((g.E + 255) / 256);
    if (nvar == 3) {
        DG_DISPATCH_N(n, hipLaunchKernelGGL((k_means<NT, 3>), dim3(blocks), dim3(256), 0, s, g, u, out));
    } else if (nvar == 4) {
        DG_DISPATCH_N(n, hipLaunchKernelGGL((k_means<NT, 4>), dim3(blocks), dim3(256), 0, s, g, u, out));
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dt(int n, const Geo& g, const double* u, const double* eq, double* dt_part, unsigned int* bad_part,
                     hipStream_t s) {
    const int blocks = dt_blocks(g);
    DG_DISPATCH_CL(g.closure, hipLaunchKernelGGL((k_dt<CT>), dim3(blocks), dim3(256), 0, s, g, n * n, u, eq, dt_part,
                                                 bad_part));
    return hipGetLastError();
}

hipError_t launch_step_begin_table(const Geo& g, StepBlock* sb, const RKTable& tab, const double* dt_part,
                                  const unsigned int* bad_part, int nblk, double* t_dev, double dt_fixed,
                                  double* dt_used, hipStream_t s) {
    if (tab.s < 1 || tab.s > kMaxStages || nblk < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_step_begin_table, dim3(1), dim3(256), 0, s, g, sb, tab, dt_part, bad_part, nblk, t_dev,
                       dt_fixed, dt_used);
    return hipGetLastError();
}

hipError_t launch_rk_combine(const double* base, const double* const* k, int nk, const double* coef,
                             double* out, long long n, hipStream_t s) {
    if (nk < 1 || nk > kMaxStages) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    KPtrs kp{};
    for (int j = 0; j < nk; ++j) {
        if (!k[j]) return hipErrorInvalidValue;
        kp.k[j] = k[j];
    }
    for (int j = nk; j < kMaxStages; ++j) kp.k[j] = k[0];
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_rk_combine, dim3((unsigned)blocks), dim3(256), 0, s, base, kp, nk, coef, out, n);
    return hipGetLastError();
}

hipError_t launch_step_begin(const Geo& g, StepBlock* sb, const double* dt_part, const unsigned int* bad_part,
                             int nblk, double* t_dev, double dt_fixed, double* dt_used, int nst, hipStream_t s) {
    if ((nst != 2 && nst != 3) || nblk < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(256), 0, s, g, sb, dt_part, bad_part, nblk, t_dev, dt_fixed,
                       dt_used, nst);
    return hipGetLastError();
}

hipError_t launch_damp_prep(int n, const Geo& g, const double* u0, const int* list, int nlist, double* q0,
                            hipStream_t s) {
    if (nlist <= 0) return hipSuccess;
    DG_DISPATCH_CL(g.closure, DG_DISPATCH_N(n, hipLaunchKernelGGL((k_damp_prep<NT, CT>), dim3(nlist), dim3(64), 0, s,
                                                                  g, u0, list, q0)));
    return hipGetLastError();
}

hipError_t launch_damp(int n, const Geo& g, double* u, const double* q0, const double* eq, const int* list,
                       int nlist, const StageCoeffs* sc, hipStream_t s, bool rev) {
    if (nlist <= 0) return hipSuccess;
    DG_DISPATCH_CL(g.closure, DG_DISPATCH_N(n, hipLaunchKernelGGL((k_damp_c<NT, CT>), dim3(nlist), dim3(64), 0, s, g,
                                                                  u, q0, eq, list, nlist, sc, rev ? 1 : 0)));
    return hipGetLastError();
}

hipError_t launch_stage_dev(int n, const Geo& g, const double* du, const double* dun, const double* du0,
                            const double* leq, const float* eqtr, double* out, const StageCoeffs* sc,
                            hipStream_t s, bool rev) {
    if (!dun) dun = du;
    if (!du0) du0 = du;
    if (!leq || !eqtr) return hipErrorInvalidValue;
    DG_DISPATCH_N(n, {
        constexpr int EW = 64 / NT;
        const int tx = (g.nx + EW - 1) / EW;
        const int tt = tx * g.ny;
        hipLaunchKernelGGL((k_stage_dev_c<NT>), dim3(tt), dim3(64), 0, s, g, tx, tt, du, dun, du0, leq, eqtr, out,
                           sc, rev ? 1 : 0);
    });
    return hipGetLastError();
}

long long eq_trace_entries(int n, const Geo& g) { return (long long)g.tiles_x * g.ny * 4 * 3 * n * (64 / n); }

hipError_t launch_eq_traces(int n, const Geo& g, const double* eq, float* eqtr, hipStream_t s) {
    const int blocks = (int)((g.E + 63) / 64);
    DG_DISPATCH_N(n, hipLaunchKernelGGL((k_eq_traces<NT>), dim3(blocks), dim3(64), 0, s, g, eq, eqtr));
    return hipGetLastError();
}

hipError_t launch_add_state(const double* a, const double* b, double* out, double sign, long long n,
                            hipStream_t s) {
    const int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_add_state, dim3(blocks), dim3(256), 0, s, a, b, out, sign, n);
    return hipGetLastError();
}

// one partial per block of four tiles
int torque_partials(const Geo& g) { return g.tiles_x * g.ny; }

hipError_t launch_torque(int n, const Geo& g, double t, const double* t_dev, const double* u, const double* eq,
                         double* partials, double* out, hipStream_t s) {
    const int np = torque_partials(g);
    const int nblocks = (np + kTorqueWaves - 1) / kTorqueWaves;
    DG_DISPATCH_N(n, hipLaunchKernelGGL((k_torque<NT>), dim3(nblocks), dim3(64 * kTorqueWaves), 0, s, g, t, t_dev, u,
                                         eq, partials));
    hipLaunchKernelGGL(k_torque_final, dim3(1), dim3(kTorqueFinal), 0, s, partials, np, out);
    return hipGetLastError();
}

hipError_t launch_torque_final(const Geo& g, const double* partials, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_torque_final, dim3(1), dim3(kTorqueFinal), 0, s, partials, torque_partials(g), out);
    return hipGetLastError();
}

}  // namespace dgk
