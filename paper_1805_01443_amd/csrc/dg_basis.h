// Compile-time Gauss-Legendre rules and Legendre basis tables for n = 2..5
// points (Sec. 2.2: modal Legendre basis, Gauss-Legendre quadrature of eq. (3)).
// Evaluated as constant expressions, so kernels templated on n see every table
// entry as an immediate constant; the host uses the same values.
#pragma once

namespace dgk {

constexpr int kMaxOrder = 5;

// square root by Newton's iteration from above (constant-expression safe)
constexpr double csqrt(double x) {
    if (x <= 0.0) return 0.0;
    double r = x > 1.0 ? x : 1.0;
    for (int it = 0; it < 200; ++it) {
        const double nr = 0.5 * (r + x / r);
        if (!(nr < r)) break;
        r = nr;
    }
    return r;
}

// Legendre P_a(x) and P_a'(x) by the three-term recurrences
constexpr double cleg(int a, double x) {
    double p0 = 1.0, p1 = x;
    if (a == 0) return 1.0;
    for (int k = 1; k < a; ++k) {
        const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

constexpr double cdleg(int a, double x) {
    // P'_{k+1} = P'_{k-1} + (2k+1) P_k
    if (a == 0) return 0.0;
    double dm1 = 0.0, d0 = 1.0;
    for (int k = 1; k < a; ++k) {
        const double d1 = dm1 + (2.0 * k + 1.0) * cleg(k, x);
        dm1 = d0;
        d0 = d1;
    }
    return d0;
}

struct BasisTab {
    double xi[kMaxOrder];              // nodes, ascending
    double wh[kMaxOrder];              // weights / 2 (sum 1)
    double phi[kMaxOrder][kMaxOrder];  // phi_a(xi_q)
    double dphi[kMaxOrder][kMaxOrder]; // phi_a'(xi_q)
    double wphi[kMaxOrder][kMaxOrder]; // wh_q phi_a(xi_q)
    double wdphi[kMaxOrder][kMaxOrder];// wh_q phi_a'(xi_q)
    double pm[kMaxOrder], pp[kMaxOrder];  // phi_a(-1), phi_a(+1)
    double D[kMaxOrder][kMaxOrder];    // D[a][c] = (1/2) int phi_a' phi_c
};

// closed-form Gauss-Legendre rules (positive nodes and their weights)
constexpr BasisTab make_basis(int n) {
    BasisTab t{};
    double x[kMaxOrder] = {}, w[kMaxOrder] = {};
    if (n == 2) {
        const double a = csqrt(1.0 / 3.0);
        x[0] = -a; x[1] = a;
        w[0] = 1.0; w[1] = 1.0;
    } else if (n == 3) {
        const double a = csqrt(3.0 / 5.0);
        x[0] = -a; x[1] = 0.0; x[2] = a;
        w[0] = 5.0 / 9.0; w[1] = 8.0 / 9.0; w[2] = 5.0 / 9.0;
    } else if (n == 4) {
        const double s = 2.0 / 7.0 * csqrt(6.0 / 5.0);
        const double a = csqrt(3.0 / 7.0 - s), b = csqrt(3.0 / 7.0 + s);
        const double s30 = csqrt(30.0);
        x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
        w[0] = (18.0 - s30) / 36.0; w[1] = (18.0 + s30) / 36.0;
        w[2] = w[1]; w[3] = w[0];
    } else if (n == 5) {
        const double s = 2.0 * csqrt(10.0 / 7.0);
        const double a = csqrt(5.0 - s) / 3.0, b = csqrt(5.0 + s) / 3.0;
        const double s70 = csqrt(70.0);
        x[0] = -b; x[1] = -a; x[2] = 0.0; x[3] = a; x[4] = b;
        w[0] = (322.0 - 13.0 * s70) / 900.0; w[1] = (322.0 + 13.0 * s70) / 900.0;
        w[2] = 128.0 / 225.0; w[3] = w[1]; w[4] = w[0];
    }
    for (int q = 0; q < n; ++q) {
        t.xi[q] = x[q];
        t.wh[q] = 0.5 * w[q];
    }
    for (int a = 0; a < n; ++a) {
        const double s = csqrt(2.0 * a + 1.0);
        for (int q = 0; q < n; ++q) {
            t.phi[a][q] = s * cleg(a, x[q]);
            t.dphi[a][q] = s * cdleg(a, x[q]);
            t.wphi[a][q] = t.wh[q] * t.phi[a][q];
            t.wdphi[a][q] = t.wh[q] * t.dphi[a][q];
        }
        t.pp[a] = s;
        t.pm[a] = (a % 2) ? -s : s;
    }
    // (1/2) int_{-1}^{1} phi_a' phi_c = sqrt((2a+1)(2c+1)) for a > c with a + c
    // odd, else 0 (the degree-(a-1) derivative is orthogonal to higher c)
    for (int a = 0; a < n; ++a)
        for (int c = 0; c < n; ++c)
            t.D[a][c] = (a > c && ((a + c) % 2 == 1)) ? csqrt((2.0 * a + 1.0) * (2.0 * c + 1.0)) : 0.0;
    return t;
}

template <int N>
struct Basis {
    static constexpr BasisTab t = make_basis(N);
};

// Gauss-Lobatto rule of the positivity limiter (Sec. 2.4, after Zhang & Shu):
// the fewest points L with 2L - 3 >= N_p, closed forms for L = 2..4 (which
// covers n <= 5); w1h = half the end weight of the rule normalised to sum 1.
struct LobattoTab {
    int L;
    double x[kMaxOrder];
    double w1h;
    double phi[kMaxOrder][kMaxOrder];  // phi_a(x_q)
};

constexpr LobattoTab make_lobatto(int n) {
    LobattoTab t{};
    int L = 2;
    while (2 * L - 3 < n - 1) ++L;
    t.L = L;
    if (L == 2) {
        t.x[0] = -1.0; t.x[1] = 1.0;
        t.w1h = 0.5 * 0.5;
    } else if (L == 3) {
        t.x[0] = -1.0; t.x[1] = 0.0; t.x[2] = 1.0;
        t.w1h = 0.5 / 6.0;
    } else {
        const double a = 1.0 / csqrt(5.0);
        t.x[0] = -1.0; t.x[1] = -a; t.x[2] = a; t.x[3] = 1.0;
        t.w1h = 0.5 / 12.0;
    }
    for (int a = 0; a < n; ++a)
        for (int q = 0; q < L; ++q) t.phi[a][q] = csqrt(2.0 * a + 1.0) * cleg(a, t.x[q]);
    return t;
}

template <int N>
struct Lobatto {
    static constexpr LobattoTab t = make_lobatto(N);
};

}  // namespace dgk
