// Host computation of the lattice constants and the polynomial-equilibrium
// coefficients from their closed forms, in long double.
//
//  * Riemann zeta at 3, 3/2, 5/2, 7/2 through the Dirichlet eta function,
//    zeta(s) = eta(s) / (1 - 2^(1-s)), with eta summed by P. Borwein's
//    accelerated alternating-series algorithm ("An efficient algorithm for the
//    Riemann zeta function", 2000), n = 40 terms (error ~ (3 + sqrt 8)^-40).
//  * Cubature at mu0 = 0: Eq. QuadSolution2Dmu0 (d = 2) and
//    Eq. QuadSolution3Dmu0 (d = 3); weights by class from Eqs. QuadSolution2D /
//    QuadSolution3D; xi = xi(beta0 = 1) / sqrt(beta0).
//  * alpha_1..alpha_5: Appendix (d = 2 and d = 3); alpha_1 and alpha_2 are
//    affine in b = beta0 eps_FD.
#pragma once

#include <cmath>

namespace mlbm {

struct HostConst {
    double a;          // weight parameter
    double xi1;        // xi at beta0 = 1
    double wcls[3];    // weight of a velocity with 0, 1, 2 nonzero components
    double a1_0, a1_b, a2_0, a2_b, a3, a4, a5;
};

inline long double eta_borwein(long double s) {
    constexpr int n = 40;
    long double d[n + 1];
    long double term = 1.0L / n;   // i = 0: (n-1)! / n!
    long double acc = term;
    d[0] = n * acc;
    for (int i = 1; i <= n; ++i) {
        term *= 4.0L * (n + i - 1) * (n - i + 1) / ((2.0L * i - 1.0L) * (2.0L * i));
        acc += term;
        d[i] = n * acc;
    }
    long double sum = 0.0L;
    for (int k = 0; k < n; ++k) {
        const long double t = (d[k] - d[n]) / powl(static_cast<long double>(k + 1), s);
        sum += (k & 1) ? -t : t;
    }
    return -sum / d[n];
}

inline long double zeta_ld(long double s) { return eta_borwein(s) / (1.0L - powl(2.0L, 1.0L - s)); }

inline HostConst host_constants(int d) {
    const long double pi = 3.14159265358979323846264338327950288L;
    const long double ln2 = 0.69314718055994530941723212145817657L;
    const long double s2 = sqrtl(2.0L);
    HostConst h{};
    if (d == 2) {
        const long double z3 = zeta_ld(3.0L);
        const long double a = powl(pi, 4) / (972.0L * z3 * ln2);
        const long double xi1 = (3.0L / pi) * sqrtl(3.0L * z3);
        const long double fac = 72.0L * ln2 / (216.0L * ln2 * z3 - powl(pi, 4));
        const long double p6 = pi * pi / 6.0L;
        h.a = static_cast<double>(a);
        h.xi1 = static_cast<double>(xi1);
        h.wcls[0] = static_cast<double>(1.0L - 5.0L * a);
        h.wcls[1] = static_cast<double>(a);
        h.wcls[2] = static_cast<double>(a / 4.0L);
        h.a1_0 = static_cast<double>(fac * 3.0L * z3);
        h.a1_b = static_cast<double>(-fac * p6);
        h.a2_0 = static_cast<double>(-fac * p6);
        h.a2_b = static_cast<double>(fac * 2.0L * ln2);
        h.a3 = static_cast<double>(12.0L * ln2 / (pi * pi));
        h.a4 = static_cast<double>(fac * ln2);
        h.a5 = static_cast<double>(-fac * p6);
    } else {
        const long double z32 = zeta_ld(1.5L), z52 = zeta_ld(2.5L), z72 = zeta_ld(3.5L);
        const long double a = (41.0L + 9.0L * s2) * z52 * z52 / (558.0L * z32 * z72);
        const long double xi1 = sqrtl(3.0L * (15.0L + 2.0L * s2) * z72 / (14.0L * z52));
        const long double fac =
            4.0L * z32 / (5.0L * (9.0L - 5.0L * s2) * z32 * z72 - 3.0L * (9.0L - 4.0L * s2) * z52 * z52);
        h.a = static_cast<double>(a);
        h.xi1 = static_cast<double>(xi1);
        h.wcls[0] = static_cast<double>(1.0L - 12.0L * a);
        h.wcls[1] = static_cast<double>(a);
        h.wcls[2] = static_cast<double>(a / 2.0L);
        h.a1_0 = static_cast<double>(fac * 1.25L * (9.0L - 5.0L * s2) * z72);
        h.a1_b = static_cast<double>(-fac * (5.0L - 3.0L * s2) * z52);
        h.a2_0 = static_cast<double>(-fac * (5.0L - 3.0L * s2) * z52);
        h.a2_b = static_cast<double>(fac * (6.0L - 4.0L * s2) * z32 * (2.0L / 3.0L));
        h.a3 = static_cast<double>(2.0L * z32 / ((3.0L + s2) * z52));
        h.a4 = static_cast<double>(fac * (3.0L - 2.0L * s2) * z32);
        h.a5 = static_cast<double>(-fac * (5.0L - 3.0L * s2) * z52);
    }
    return h;
}

// n-point Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on
// the Legendre polynomial (three-term recurrence).
inline void gauss_legendre(int n, double* x, double* w) {
    const long double pi = 3.14159265358979323846264338327950288L;
    for (int i = 0; i < n; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
        long double dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            const long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = static_cast<double>(z);
        w[i] = static_cast<double>(2.0L / ((1.0L - z * z) * dp * dp));
    }
}

}  // namespace mlbm
