// Zhang-Shu positivity factors of one element (Sec. 2.4), shared by the
// positivity kernel (rows loaded from the state) and the stage kernel with the
// scaling fused (rows still in registers).  N lanes per element: lane k holds
// mode row k of every variable, Ua[v][b] = u[v][k][b].
//
// Test points: Lobatto x Gauss and Gauss x Lobatto (L Lobatto points with
// 2L - 3 >= the polynomial degree).  theta1 brings the smallest point density
// up to eps; theta2 is the smallest admissible t in [0, 1] of the pressure of
// mean + t (point - mean), with the density already limited, found by 64
// bisection steps that keep the admissible end (p is concave along the
// segment); each step tests rho p >= eps rho, the density on the segment
// being positive.  eps = min(e0, mean density, mean pressure).  An element whose
// mean is not admissible keeps theta1 = theta2 = 1.
#pragma once

#include "dg_basis.h"
#include "dg_internal.h"

namespace dgk {

// LDS entries per element slot: rows at the Gauss and at the Lobatto y
// points, the means and two per-lane minima
template <int N, int NV>
constexpr int pp_slot() {
    return NV * N * N + NV * N * Lobatto<N>::t.L + NV + 2 * N;
}

// theta1 (density) and theta2 (pressure) of the element; S is the element's
// slot (pp_slot doubles), k the lane's index in the element.  Every lane of
// the wavefront calls it (it holds barriers); a lane of an idle slot works on
// a valid element and its results go unused.
template <int N, int NV>
__device__ __forceinline__ void pp_factors(const Geo& g, double* S, int k, const double (&Ua)[NV][N], double e0,
                                           double& th1, double& th2) {
    constexpr auto& G = Basis<N>::t;
    constexpr auto& Lb = Lobatto<N>::t;
    constexpr int L = Lb.L;
    constexpr int SA = NV * N * N;  // [v][a][r]: row a at Gauss eta_r
    constexpr int SB = NV * N * L;  // [v][a][r]: row a at Lobatto eta_r
    constexpr int NP = N + L;       // test points per lane (the first N need k < L)
    // row k contracted in y at the Gauss and at the Lobatto points
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double c = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) c = fma(Ua[v][b], G.phi[b][r], c);
            S[(v * N + k) * N + r] = c;
        }
#pragma unroll
        for (int r = 0; r < L; ++r) {
            double c = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) c = fma(Ua[v][b], Lb.phi[b][r], c);
            S[SA + (v * N + k) * L + r] = c;
        }
        if (k == 0) S[SA + SB + v] = Ua[v][0];  // the mean
    }
    __syncthreads();
    double M[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) M[v] = S[SA + SB + v];
    const bool adi = NV == 4 && g.closure == 2;
    const double gm1 = g.gamma - 1.0;
    double pbar = M[0];
    if (adi) pbar = gm1 * (M[3] - 0.5 * (M[1] * M[1] + M[2] * M[2]) / M[0]);
    const bool admissible = M[0] > 0.0 && pbar > 0.0;
    double eps = e0;
    if (M[0] < eps) eps = M[0];
    if (adi && pbar < eps) eps = pbar;
    // basis values phi_a(x_k) at this lane's Lobatto and Gauss x
    double pl[N], pg[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        double x = Lb.phi[a][0], y = G.phi[a][0];
#pragma unroll
        for (int m = 1; m < N; ++m) {
            if (m < L) x = k == m ? Lb.phi[a][m] : x;
            y = k == m ? G.phi[a][m] : y;
        }
        pl[a] = x;
        pg[a] = y;
    }
    const bool hasA = k < L;
    // value of variable v at this lane's test point p (p < N: (Lobatto x_k,
    // Gauss eta_p); else (Gauss x_k, Lobatto eta_{p-N}))
    auto point = [&](int v, int p) __attribute__((always_inline)) {
        double s2 = 0.0;
        if (p < N) {
#pragma unroll
            for (int a = 0; a < N; ++a) s2 = fma(pl[a], S[(v * N + a) * N + p], s2);
        } else {
#pragma unroll
            for (int a = 0; a < N; ++a) s2 = fma(pg[a], S[SA + (v * N + a) * L + (p - N)], s2);
        }
        return s2;
    };
    double rmin = INFINITY;
#pragma unroll
    for (int p = 0; p < NP; ++p)
        if (p >= N || hasA) rmin = fmin(rmin, point(0, p));
    // element minimum over its N lanes
    S[SA + SB + NV + k] = rmin;
    __syncthreads();
    double emin = INFINITY;
#pragma unroll
    for (int m = 0; m < N; ++m) emin = fmin(emin, S[SA + SB + NV + m]);
    th1 = 1.0;
    th2 = 1.0;
    if (admissible && emin < eps) th1 = (M[0] - eps) / (M[0] - emin);
    if (adi) {
        // the points whose density-limited value has p < eps, as a bit list
        unsigned need = 0u;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (!admissible || (p < N && !hasA)) continue;
            const double w0 = M[0] + th1 * (point(0, p) - M[0]);
            const double w1 = point(1, p), w2 = point(2, p), w3 = point(NV - 1, p);
            const double pw = gm1 * (w3 - 0.5 * (w1 * w1 + w2 * w2) / w0);
            if (pw < eps) need |= 1u << p;
        }
        // Each lane works through its own list, two points at a time: two
        // independent bisections in flight, and a wavefront takes as many
        // rounds as its longest list needs, not one per point any lane needs.
        // The values and every step are those of a bisection of one point, so
        // theta2 (the minimum over the points) keeps its bits.
        while (__any(need != 0u)) {
            const int p1 = need ? __builtin_ctz(need) : 0;
            const bool h1 = need != 0u;
            need &= need - 1u;
            const int p2 = need ? __builtin_ctz(need) : p1;
            const bool h2 = need != 0u;
            need &= need - 1u;
            // value of variable v at point q (run-time index), as point() does
            auto at = [&](int v, int q) __attribute__((always_inline)) {
                double s2 = 0.0;
                const bool ga = q < N;
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const int ix = ga ? (v * N + a) * N + q : SA + (v * N + a) * L + (q - N);
                    s2 = fma(ga ? pl[a] : pg[a], S[ix], s2);
                }
                return s2;
            };
            const double a0 = M[0] + th1 * (at(0, p1) - M[0]);
            const double a1 = at(1, p1), a2 = at(2, p1), a3 = at(NV - 1, p1);
            const double b0 = M[0] + th1 * (at(0, p2) - M[0]);
            const double b1 = at(1, p2), b2 = at(2, p2), b3 = at(NV - 1, p2);
            double lo1 = 0.0, hi1 = 1.0, lo2 = 0.0, hi2 = 1.0;
            for (int it = 0; it < 64; ++it) {
                const double m1 = 0.5 * (lo1 + hi1), m2 = 0.5 * (lo2 + hi2);
                const double s0 = M[0] + m1 * (a0 - M[0]), s1 = M[1] + m1 * (a1 - M[1]);
                const double s2 = M[2] + m1 * (a2 - M[2]), s3 = M[NV - 1] + m1 * (a3 - M[NV - 1]);
                const double t0 = M[0] + m2 * (b0 - M[0]), t1 = M[1] + m2 * (b1 - M[1]);
                const double t2 = M[2] + m2 * (b2 - M[2]), t3 = M[NV - 1] + m2 * (b3 - M[NV - 1]);
                // rho p >= eps rho (the density on the segment is positive):
                // no division in the loop
                const double ps = gm1 * (s3 * s0 - 0.5 * (s1 * s1 + s2 * s2));
                const double pt = gm1 * (t3 * t0 - 0.5 * (t1 * t1 + t2 * t2));
                if (ps >= eps * s0)
                    lo1 = m1;
                else
                    hi1 = m1;
                if (pt >= eps * t0)
                    lo2 = m2;
                else
                    hi2 = m2;
            }
            if (h1) th2 = fmin(th2, lo1);
            if (h2) th2 = fmin(th2, lo2);
        }
        // element minimum over its N lanes (adi is uniform: no divergent barrier)
        S[SA + SB + NV + N + k] = th2;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < N; ++m) th2 = fmin(th2, S[SA + SB + NV + N + m]);
    }
}

// the row scaled: density by theta1, then every variable by theta2; the
// mean (mode (0, 0), lane 0's b = 0) never changes.  Factors of 1 leave the
// row bit for bit.
template <int N, int NV>
__device__ __forceinline__ void pp_scale_row(int k, double th1, double th2, double (&Ua)[NV][N]) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const double x = Ua[v][b];
            double y = x;
            if (v == 0) y *= th1;
            y *= th2;
            Ua[v][b] = (b == 0 && k == 0) ? x : y;  // a value select: no branch per lane
        }
}

}  // namespace dgk
