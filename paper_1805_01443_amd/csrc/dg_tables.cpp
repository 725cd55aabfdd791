// Host-side quadrature and basis tables (Sec. 2.2: Gauss-Legendre points for
// the volume and edge integrals of eq. (3); Legendre modal basis), generated
// once per handle in FP64 and handed to the kernels by value.
#include <cmath>

#include "dg_internal.h"

namespace dgk {

namespace {

// P_n(x) and P_{n-1}(x) by the three-term recurrence
void legendre_pair(int n, double x, double* pn, double* pn1) {
    double a = 1.0, b = x;  // P_0, P_1
    if (n == 0) {
        *pn = 1.0;
        *pn1 = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    *pn = b;
    *pn1 = a;
}

double legendre(int n, double x) {
    double p, q;
    legendre_pair(n, x, &p, &q);
    return p;
}

// derivative from the closed form P_n' = n (x P_n - P_{n-1}) / (x^2 - 1) away
// from the end points, and P_n'(+-1) = (+-1)^(n+1) n (n+1) / 2 there
double legendre_d(int n, double x) {
    if (n == 0) return 0.0;
    if (std::fabs(std::fabs(x) - 1.0) < 1e-300) {
        double s = (x > 0 || (n % 2 == 1)) ? 1.0 : -1.0;
        return s * 0.5 * n * (n + 1);
    }
    double p, q;
    legendre_pair(n, x, &p, &q);
    return n * (x * p - q) / (x * x - 1.0);
}

}  // namespace

double basis_phi(int a, double x) { return std::sqrt(2.0 * a + 1.0) * legendre(a, x); }

int make_tables(int n, Tables* t) {
    if (n < 1 || n > kMaxN) return -1;
    *t = Tables{};
    const double pi = 3.141592653589793238462643;
    for (int k = 0; k < n; ++k) {
        // Tricomi's asymptotic first guess for the k-th largest root, then Newton
        double th = pi * (4.0 * k + 3.0) / (4.0 * n + 2.0);
        double z = std::cos(th) * (1.0 - (1.0 - 1.0 / n) / (8.0 * n * n));
        for (int it = 0; it < 60; ++it) {
            double p, q;
            legendre_pair(n, z, &p, &q);
            double dp = n * (z * p - q) / (z * z - 1.0);
            double dz = p / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16 * std::fabs(z) + 1e-300) break;
        }
        if (2 * k + 1 == n) z = 0.0;
        double p, q;
        legendre_pair(n, z, &p, &q);
        // weight 2 (1 - z^2) / (n P_{n-1}(z))^2
        double w = 2.0 * (1.0 - z * z) / ((n * q) * (n * q));
        t->xi[n - 1 - k] = z;
        t->wh[n - 1 - k] = 0.5 * w;
    }
    // enforce exact symmetry of the rule
    for (int k = 0; k < n / 2; ++k) {
        double z = 0.5 * (t->xi[n - 1 - k] - t->xi[k]);
        double w = 0.5 * (t->wh[n - 1 - k] + t->wh[k]);
        t->xi[n - 1 - k] = z;
        t->xi[k] = -z;
        t->wh[n - 1 - k] = w;
        t->wh[k] = w;
    }
    for (int a = 0; a < n; ++a) {
        double s = std::sqrt(2.0 * a + 1.0);
        for (int q = 0; q < n; ++q) {
            t->phi[a][q] = s * legendre(a, t->xi[q]);
            t->dphi[a][q] = s * legendre_d(a, t->xi[q]);
        }
        t->pp[a] = s;
        t->pm[a] = (a % 2) ? -s : s;
    }
    return 0;
}

}  // namespace dgk
