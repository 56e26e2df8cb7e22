// Complete Fermi-Dirac integrals F_k(x) in double precision on the device,
// and the inversion of the channel density n = (2 pi / beta)^(d/2)
// F_{d/2-1}(nu) (Sec. 2.2, Eqs. nFDstdOmega and energyFDstdOmega).
//
// F_k(x) = Gamma(k+1)^-1 int_0^inf y^k / (e^(y-x) + 1) dy = -Li_{k+1}(-e^x),
// dF_k/dx = F_{k-1}, F_{-1} = logistic, F_0 = log(1 + e^x) (Sec. 2.2).
//
// Methods (chosen here; the paper defers to the literature):
//  * x <= -1: the polylogarithm series sum_j (-1)^(j+1) e^(j x) / j^(k+1),
//    truncated when a term falls below 1e-18 of the sum (at most 60 terms).
//  * half-integer k = m - 1/2, x > -1: with y = t^2 the integrand
//    2 t^(2m) / (e^(t^2 - x) + 1) is even and analytic in the strip
//    |Im t| < Im sqrt(x + i pi), so the trapezoidal rule on the half line
//    converges geometrically; the step is 0.12 times that strip half-width
//    (error ~ exp(-2 pi / 0.12)).  Supported for x <= 4000.
//  * F_1 (d = 2 energy), x > -1: for x >= 1 the exact reflection
//    F_1(x) = pi^2/6 + x^2/2 - F_1(-x); for -1 < x < 1,
//    F_1(x) = F_1(-1) + int_{-1}^{x} F_0(s) ds by 20-point Gauss-Legendre
//    (F_0 is analytic in a strip of half-width pi around the real axis).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace mlbm {
namespace fd {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;

__device__ __forceinline__ double logistic(double z) {
    if (z >= 0.0) return 1.0 / (1.0 + exp(-z));
    const double e = exp(z);
    return e / (1.0 + e);
}

// j^(-s) for s = TWO_S / 2 and j = 1..60, tabulated at compile time (square
// roots by Newton's iteration to its fixed point) so that the series below
// spend no division or square root per term.
constexpr double const_sqrt(double x) {
    double g = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 200; ++i) {
        const double n = 0.5 * (g + x / g);
        if (n == g) break;
        g = n;
    }
    return g;
}

constexpr int kSeriesTerms = 60;

template <int TWO_S>
struct JpowTable {
    double v[kSeriesTerms + 1];
    constexpr JpowTable() : v() {
        for (int j = 1; j <= kSeriesTerms; ++j) {
            double p = 1.0;
            for (int r = 0; r < TWO_S / 2; ++r) p *= j;
            if (TWO_S & 1) p *= const_sqrt(static_cast<double>(j));
            v[j] = 1.0 / p;
        }
    }
};

__constant__ const JpowTable<1> kJpow1{};
__constant__ const JpowTable<3> kJpow3{};
__constant__ const JpowTable<4> kJpow4{};
__constant__ const JpowTable<5> kJpow5{};
__constant__ const JpowTable<7> kJpow7{};

template <int TWO_S>
__device__ __forceinline__ double jpow_inv(int j) {
    static_assert(TWO_S == 1 || TWO_S == 3 || TWO_S == 4 || TWO_S == 5 || TWO_S == 7, "no table for this order");
    if constexpr (TWO_S == 1) return kJpow1.v[j];
    else if constexpr (TWO_S == 3) return kJpow3.v[j];
    else if constexpr (TWO_S == 4) return kJpow4.v[j];
    else if constexpr (TWO_S == 5) return kJpow5.v[j];
    else return kJpow7.v[j];
}

// sum_{j>=1} (-1)^(j+1) e^(j x) / j^s, s = TWO_S / 2, for x <= -1.
template <int TWO_S>
__device__ double series(double x) {
    const double t = exp(x);
    double pj = t, sum = 0.0;
    for (int j = 1; j <= kSeriesTerms; ++j) {
        const double term = pj * jpow_inv<TWO_S>(j);
        sum += (j & 1) ? term : -term;
        if (term <= 1e-18 * sum) break;
        pj *= t;
    }
    return sum;
}

// Two series of the same argument in one pass (shared powers of e^x).
template <int TWO_A, int TWO_B>
__device__ void series_pair(double x, double& sa, double& sb) {
    const double t = exp(x);
    double pj = t;
    sa = 0.0;
    sb = 0.0;
    for (int j = 1; j <= kSeriesTerms; ++j) {
        const double ta = pj * jpow_inv<TWO_A>(j), tb = pj * jpow_inv<TWO_B>(j);
        sa += (j & 1) ? ta : -ta;
        sb += (j & 1) ? tb : -tb;
        if (ta <= 1e-18 * sa && tb <= 1e-18 * sb) break;
        pj *= t;
    }
}

// Three series of the same argument in one pass.
template <int TWO_A, int TWO_B, int TWO_C>
__device__ void series_triple(double x, double& sa, double& sb, double& sc) {
    const double t = exp(x);
    double pj = t;
    sa = 0.0;
    sb = 0.0;
    sc = 0.0;
    for (int j = 1; j <= kSeriesTerms; ++j) {
        const double ta = pj * jpow_inv<TWO_A>(j), tb = pj * jpow_inv<TWO_B>(j), tc = pj * jpow_inv<TWO_C>(j);
        sa += (j & 1) ? ta : -ta;
        sb += (j & 1) ? tb : -tb;
        sc += (j & 1) ? tc : -tc;
        if (ta <= 1e-18 * sa && tb <= 1e-18 * sb && tc <= 1e-18 * sc) break;
        pj *= t;
    }
}

// Reversion of the series F_{1/2}(x) = sum_j (-1)^(j+1) z^j / j^(3/2), z = e^x:
// z = sum_{n=1..kRev} g_n c^n solves F_{1/2}(x) = c up to O(c^(kRev+1)).  The
// g_n follow by composing term by term: with g_1 = 1, g_n is minus the c^n
// coefficient of f(g(c)) computed with g_n = 0 (computed at compile time).
constexpr int kRev = 8;
struct HalfReversion {
    double g[kRev + 1];
    constexpr HalfReversion() : g() {
        double f[kRev + 1] = {};
        for (int j = 1; j <= kRev; ++j) f[j] = ((j & 1) ? 1.0 : -1.0) / (j * const_sqrt(static_cast<double>(j)));
        g[1] = 1.0;
        for (int n = 2; n <= kRev; ++n) {
            double cur[kRev + 1] = {};          // g(c)^m, truncated at degree kRev
            for (int q = 1; q <= kRev; ++q) cur[q] = g[q];
            double acc = 0.0;
            for (int m = 1; m <= n; ++m) {
                acc += f[m] * cur[n];
                double nxt[kRev + 1] = {};
                for (int a = 1; a <= kRev; ++a)
                    for (int b = 1; a + b <= kRev; ++b) nxt[a + b] += cur[a] * g[b];
                for (int q = 0; q <= kRev; ++q) cur[q] = nxt[q];
            }
            g[n] = -acc;
        }
    }
};
__constant__ const HalfReversion kHalfRev{};

// F_{M - 1/2}(x) by the trapezoidal rule described above, x > -1.
// Arguments above kXMax (or NaN) return NaN: the step count grows like x,
// and such degenerate states are outside the supported range.
constexpr double kXMax = 4000.0;

template <int M>
__device__ double half_quad(double x) {
    if (!(x <= kXMax)) return __builtin_nan("");
    const double a = sqrt(0.5 * (sqrt(x * x + kPi * kPi) - x));
    const double h = 0.12 * a;
    const double tmax = sqrt(fmax(x, 0.0) + 50.0);
    const int n = static_cast<int>(ceil(tmax / h));
    double s = (M == 0) ? 0.5 * logistic(x) : 0.0;
    for (int j = 1; j <= n; ++j) {
        const double t = j * h;
        const double t2 = t * t;
        double pw = 1.0;
#pragma unroll
        for (int r = 0; r < M; ++r) pw *= t2;
        s += pw * logistic(x - t2);
    }
    // Gamma(M + 1/2) = sqrt(pi) (2M)! / (4^M M!)
    double g = kSqrtPi;
#pragma unroll
    for (int r = 1; r <= M; ++r) g *= (r - 0.5);
    return 2.0 * h * s / g;
}

// F_{M - 1/2}(x), M = 0..3.
template <int M>
__device__ __forceinline__ double half(double x) {
    return (x <= -1.0) ? series<2 * M + 1>(x) : half_quad<M>(x);
}

__device__ __forceinline__ double F0(double x) {
    return (x <= 0.0) ? log1p(exp(x)) : x + log1p(exp(-x));
}

__device__ double F1(double x, const FdParams& fp) {
    if (x <= -1.0) return series<4>(x);
    if (x >= 1.0) return kPi * kPi / 6.0 + 0.5 * x * x - series<4>(-x);
    // F_1(-1) + int_{-1}^{x} F_0(s) ds
    const double half_len = 0.5 * (x + 1.0), mid = 0.5 * (x - 1.0);
    double s = 0.0;
    for (int j = 0; j < kGL; ++j) s += fp.gl_w[j] * F0(mid + half_len * fp.gl_x[j]);
    return series<4>(-1.0) + half_len * s;
}

// nu with F_{1/2}(nu) = c (c > 0), Newton with F_{-1/2} as derivative.
// F_{1/2} is increasing and convex, so after at most one overshoot the
// iterates approach the root monotonically.  Returns false on failure.
__device__ bool invert_half(double c, double& nu) {
    nu = (c < 1.0) ? log(c) : pow(c * 1.32934038817913702047, 2.0 / 3.0);  // Gamma(5/2) c
    for (int it = 0; it < 60; ++it) {
        const double f = half<1>(nu) - c;
        const double d = f / half<0>(nu);
        nu -= d;
        if (!isfinite(nu)) return false;
        if (fabs(d) <= 2e-15 * fmax(1.0, fabs(nu))) return true;
    }
    return false;
}

// nu = beta mu of a channel with density n at inverse temperature beta.
template <int D>
__device__ __forceinline__ bool channel_nu(double n, double beta, double& nu) {
    if constexpr (D == 2) {
        nu = log(expm1(n * beta / (2.0 * kPi)));       // F_0 has a closed-form inverse
        return isfinite(nu);
    } else {
        const double s = beta / (2.0 * kPi);
        return invert_half(n * s * sqrt(s), nu);
    }
}

// n_{d,beta,mu} = (2 pi / beta)^(d/2) F_{d/2-1}(nu), nu = beta mu (Eq. nFDstdOmega).
template <int D>
__device__ __forceinline__ double channel_density(double beta, double nu) {
    const double s = 2.0 * kPi / beta;
    if constexpr (D == 2) return s * F0(nu);
    else return s * sqrt(s) * half<1>(nu);
}

// Isothermal model: eps_FD at inverse temperature beta of the channel
// densities n_up, n_dn (Eq. nFDstdOmega inverted, then Eq. energyFDstdOmega).
// With c = F_{d/2-1}(nu) = n (beta / 2 pi)^(d/2) known exactly, the
// denominator needs no evaluation: eps = (d/2) sum F_{d/2}(nu) / (beta sum c).
// 2D: nu = log(expm1(c)) in closed form.  3D: Newton on F_{1/2}(nu) = c with
// F_{1/2} and F_{-1/2} from one series pass, started at the dilute expansion
// nu = log c + c / 2^(3/2) (F_{1/2} = e^nu - e^(2 nu) / 2^(3/2) + ...).
__device__ __forceinline__ bool invert_half_fast(double c, double& nu) {
    nu = (c < 0.5) ? log(c) + 0.35355339059327376220 * c : (c < 1.0 ? log(c) : pow(c * 1.32934038817913702047, 2.0 / 3.0));
    for (int it = 0; it < 60; ++it) {
        double f, df;
        if (nu <= -1.0) series_pair<3, 1>(nu, f, df);
        else { f = half<1>(nu); df = half<0>(nu); }
        const double d = (f - c) / df;
        nu -= d;
        if (!isfinite(nu)) return false;
        if (fabs(d) <= 2e-15 * fmax(1.0, fabs(nu))) return true;
    }
    return false;
}

// Dilute 3D channel (c = F_{1/2}(nu) <= 0.2, so nu <= -1.5): F_{3/2}(nu) with
// few series passes.  The reversed series starts Newton within ~1e-15 of the
// root; each Newton step takes one pass that sums F_{3/2}, F_{1/2} and
// F_{-1/2} together.  Once a step d is below 1e-8 (the next one would be of
// order d^2), it is taken and F_{3/2} follows it to first order,
// F_{3/2}(nu - d) = F_{3/2}(nu) - d F_{1/2}(nu) + O(d^2).  False if the
// iterate leaves the series range or does not settle.
__device__ __forceinline__ bool iso_half_dilute(double c, double& f32) {
    double z = kHalfRev.g[kRev];
    for (int q = kRev - 1; q >= 1; --q) z = z * c + kHalfRev.g[q];
    double nu = log(z * c);
    for (int it = 0; it < 8; ++it) {
        if (!(nu <= -1.0)) return false;
        double f5, f3, f1;
        series_triple<5, 3, 1>(nu, f5, f3, f1);
        const double d = (f3 - c) / f1;
        nu -= d;
        if (fabs(d) <= 1e-8 * fmax(1.0, fabs(nu))) {
            f32 = f5 - d * f3;
            return isfinite(f32);
        }
    }
    return false;
}

// One channel of the isothermal energy: F_{d/2}(nu) for the channel density n
// at inverse temperature beta (NaN if the inversion fails).
template <int D>
__device__ __forceinline__ double iso_channel(double beta, double n, const FdParams& fp) {
    const double s = beta / (2.0 * kPi);
    if constexpr (D == 2) {
        return F1(log(expm1(n * s)), fp);
    } else {
        const double c = n * s * sqrt(s);
        double f32 = 0.0;
        if (c <= 0.2 && iso_half_dilute(c, f32)) return f32;
        double nu = 0.0;
        if (!invert_half_fast(c, nu)) return __builtin_nan("");
        return half<2>(nu);
    }
}

// eps_FD from the two channels' F_{d/2}(nu): (d/2) sum F_{d/2} / (beta sum c).
template <int D>
__device__ __forceinline__ double iso_energy(double beta, double n_up, double n_dn, double f_up, double f_dn) {
    const double s = beta / (2.0 * kPi);
    const double sd = (D == 2) ? s : s * sqrt(s);
    return 0.5 * D * (f_up + f_dn) / (beta * sd * (n_up + n_dn));
}

// eps_FD of Eq. energyFDstdOmega.
template <int D>
__device__ __forceinline__ double internal_energy(double beta, double nu_up, double nu_dn,
                                                  const FdParams& fp) {
    if constexpr (D == 2) {
        return (F1(nu_up, fp) + F1(nu_dn, fp)) / (beta * (F0(nu_up) + F0(nu_dn)));
    } else {
        return 1.5 * (half<2>(nu_up) + half<2>(nu_dn)) / (beta * (half<1>(nu_up) + half<1>(nu_dn)));
    }
}

}  // namespace fd
}  // namespace mlbm
