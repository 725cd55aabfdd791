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
// segment).  eps = min(e0, mean density, mean pressure).  An element whose
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
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (!admissible || (p < N && !hasA)) continue;
            // the density-limited point value (the density value again, same bits)
            const double w0 = M[0] + th1 * (point(0, p) - M[0]);
            const double w1 = point(1, p), w2 = point(2, p), w3 = point(NV - 1, p);
            const double pw = gm1 * (w3 - 0.5 * (w1 * w1 + w2 * w2) / w0);
            if (!(pw < eps)) continue;
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < 64; ++it) {
                const double mid = 0.5 * (lo + hi);
                const double s0 = M[0] + mid * (w0 - M[0]), s1 = M[1] + mid * (w1 - M[1]);
                const double s2 = M[2] + mid * (w2 - M[2]), s3 = M[NV - 1] + mid * (w3 - M[NV - 1]);
                const double ps = gm1 * (s3 - 0.5 * (s1 * s1 + s2 * s2) / s0);
                if (ps >= eps)
                    lo = mid;
                else
                    hi = mid;
            }
            th2 = fmin(th2, lo);
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
