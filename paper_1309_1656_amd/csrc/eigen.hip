// Eigen-channel form of the equilibrium (Eq. WeqDiscr taken literally), a
// checking mode of the step in double precision.
//
// Per cell, after the moments rho, u, eps (Eq. DiscrAvr):
//  1. closed-form eigen-decomposition of the Hermitian 2x2 rho: eigenvalues
//     lam_up/dn = (rho_0 +- |rho_vec|)/2, eigenvector of lam_up along
//     n = rho_vec / |rho_vec| on the Bloch sphere (remark after Prop. 1;
//     n = 0 when rho_vec = 0, where U is arbitrary and lam_up = lam_dn);
//  2. Prop. 1: find (beta, nu_up, nu_dn) with channel densities lam_s and
//     internal energy eps.  For a trial beta each nu_s follows from
//     lam_s = (2 pi / beta)^(d/2) F_{d/2-1}(nu_s); eps_FD(beta) then decreases
//     monotonically, and a Newton iteration in log(beta), safeguarded by a
//     bracket, solves eps_FD(beta) = eps, using
//       beta d eps_FD / d beta = -(1 + m) eps_FD
//                                + (m^2 / beta) sum_s F_{m-1}(nu_s)^2 / F_{m-2}(nu_s) / sum_s F_{m-1}(nu_s),
//     m = d/2 (from dF_k/dx = F_{k-1}, Sec. 2.2);
//  3. rebuild rho_eq = U diag(n_up, n_dn) U* from n_s = (2 pi/beta)^(d/2) F_{d/2-1}(nu_s)
//     and W_eq_i = w_i rho_eq P_i(u, eps_FD).
// A cell whose inversion fails gets NaN outputs, which mlbm_moments reports.
#include "common.hpp"
#include "fermi_device.hpp"
#include "internal.hpp"

namespace mlbm {

template <int D>
__device__ bool eps_of_beta(double beta, double lu, double ld, const FdParams& fp, double& e, double& bde,
                            double& nuu, double& nud) {
    if (!fd::channel_nu<D>(lu, beta, nuu) || !fd::channel_nu<D>(ld, beta, nud)) return false;
    double fm[2], fm1[2], fm2[2];
    const double nus[2] = {nuu, nud};
    for (int s = 0; s < 2; ++s) {
        if constexpr (D == 2) {
            fm[s] = fd::F1(nus[s], fp);
            fm1[s] = fd::F0(nus[s]);
            fm2[s] = fd::logistic(nus[s]);
        } else {
            fm[s] = fd::half<2>(nus[s]);
            fm1[s] = fd::half<1>(nus[s]);
            fm2[s] = fd::half<0>(nus[s]);
        }
    }
    constexpr double m = 0.5 * D;
    const double den = fm1[0] + fm1[1];
    e = m * (fm[0] + fm[1]) / (beta * den);
    bde = -(1.0 + m) * e + (m * m / beta) * (fm1[0] * fm1[0] / fm2[0] + fm1[1] * fm1[1] / fm2[1]) / den;
    return isfinite(e) && isfinite(bde);
}

template <int D>
__device__ bool fd_parameters(double lu, double ld, double eps, const FdParams& fp, double& beta, double& nuu,
                              double& nud) {
    if (!(ld > 0.0) || !(eps > 0.0)) return false;
    constexpr double m = 0.5 * D;
    double e, bde;
    double llo = log(m / eps);          // eps_FD(beta) >= eps here (F_m / F_{m-1} >= 1)
    double lhi = llo;
    bool found = false;
    for (int it = 0; it < 64; ++it) {
        lhi += 0.6931471805599453;
        if (!eps_of_beta<D>(exp(lhi), lu, ld, fp, e, bde, nuu, nud)) return false;
        if (e < eps) { found = true; break; }
        llo = lhi;
    }
    if (!found) return false;
    double L = 0.5 * (llo + lhi);
    for (int it = 0; it < 200; ++it) {
        if (!eps_of_beta<D>(exp(L), lu, ld, fp, e, bde, nuu, nud)) return false;
        const double f = e - eps;
        if (f > 0.0) llo = L;          // energy too high: beta too small
        else if (f < 0.0) lhi = L;
        else break;
        double Ln = L - f / bde;
        if (!(Ln > llo && Ln < lhi)) Ln = 0.5 * (llo + lhi);
        const double dL = Ln - L;
        L = Ln;
        if (fabs(dL) <= 1e-15 * fmax(1.0, fabs(L)) || (lhi - llo) <= 1e-15 * fmax(1.0, fabs(L))) break;
    }
    beta = exp(L);
    return eps_of_beta<D>(beta, lu, ld, fp, e, bde, nuu, nud);
}

template <int D>
__device__ __forceinline__ double channel_density(double beta, double nu, const FdParams&) {
    const double s = 2.0 * fd::kPi / beta;
    if constexpr (D == 2) return s * fd::F0(nu);
    else return s * sqrt(s) * fd::half<1>(nu);
}

template <int Q, bool PULL>
__global__ void __launch_bounds__(256)
k_step_eigen(const double* __restrict__ src, double* __restrict__ dst, const KParams p, const FdParams fp) {
    constexpr int D = Lat<Q>::D;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= p.nx || y >= p.ny) return;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const size_t row = static_cast<size_t>(z) * ny + y;
    size_t srow[Q];
    int sx[Q];
    {
        int xo[3], yo[3], zo[3] = {z, z, z};
        pull_coords(x, nx, 1, xo);
        pull_coords(y, ny, 1, yo);
        if constexpr (D == 3) pull_coords(z, nz, 1, zo);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            srow[i] = PULL ? static_cast<size_t>(zo[Lat<Q>::c(i, 2) + 1]) * ny + yo[Lat<Q>::c(i, 1) + 1] : row;
            sx[i] = PULL ? xo[Lat<Q>::c(i, 0) + 1] : x;
        }
    }
    double a[4][Q];
    double rho[4] = {0.0, 0.0, 0.0, 0.0}, J[3] = {0.0, 0.0, 0.0}, K = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            a[k][i] = src[fidx(Q, nx, srow[i], k, i, sx[i])];
            rho[k] += a[k][i];
        }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
#pragma unroll
        for (int c = 0; c < 3; ++c) J[c] += Lat<Q>::c(i, c) * a[0][i];
        K += csq<Q>(i) * a[0][i];
    }
    const double Tr = rho[0];
    double u[3], uu = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        u[c] = (c < D) ? p.xi * J[c] / Tr : 0.0;
        uu += u[c] * u[c];
    }
    const double eps = p.half_xi2 * K / Tr - 0.5 * uu;

    // 1. closed-form eigen-decomposition of rho
    const double rv = sqrt(rho[1] * rho[1] + rho[2] * rho[2] + rho[3] * rho[3]);
    const double lu = 0.5 * (Tr + rv), ld = 0.5 * (Tr - rv);
    double nhat[3] = {0.0, 0.0, 0.0};
    if (rv > 0.0) {
        for (int c = 0; c < 3; ++c) nhat[c] = rho[c + 1] / rv;
    }
    // 2. Fermi-Dirac parameters (Prop. 1)
    double beta, nuu, nud;
    const bool ok = fd_parameters<D>(lu, ld, eps, fp, beta, nuu, nud);
    // 3. rebuild rho_eq and eps_FD
    const double nu_ = channel_density<D>(beta, nuu, fp), nd_ = channel_density<D>(beta, nud, fp);
    const double eps_fd = fd::internal_energy<D>(beta, nuu, nud, fp);
    double req[4] = {nu_ + nd_, (nu_ - nd_) * nhat[0], (nu_ - nd_) * nhat[1], (nu_ - nd_) * nhat[2]};
    const double bad = ok ? 0.0 : __builtin_nan("");
    const double b = p.beta0 * eps_fd;
    const double al1 = p.a1_0 + p.a1_b * b, al2 = p.a2_0 + p.a2_b * b;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double eu = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) eu += p.xi * Lat<Q>::c(i, c) * u[c];
        const double P = al1 + al2 * p.beta0 * p.half_xi2 * csq<Q>(i) + p.a3 * p.beta0 * eu +
                         p.a4 * (p.beta0 * eu) * (p.beta0 * eu) + p.a5 * p.beta0 * 0.5 * uu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double weq = p.w[i] * req[k] * P;
            dst[fidx(Q, nx, row, k, i, x)] = a[k][i] + p.om * (weq - a[k][i]) + bad;
        }
    }
}

template <int Q>
static hipError_t eig_q(StepKind kind, const void* src, void* dst, const KParams& p, const FdParams& fp,
                        hipStream_t s) {
    dim3 blk(p.nx >= 128 ? 128 : 64, p.nx >= 128 ? 2 : 4, 1);
    dim3 grd((p.nx + blk.x - 1) / blk.x, (p.ny + blk.y - 1) / blk.y, p.nz);
    if (kind == StepKind::FusedPush || kind == StepKind::StreamOnly) return hipErrorInvalidValue;
    if (kind == StepKind::Fused)
        hipLaunchKernelGGL((k_step_eigen<Q, true>), grd, blk, 0, s, static_cast<const double*>(src),
                           static_cast<double*>(dst), p, fp);
    else
        hipLaunchKernelGGL((k_step_eigen<Q, false>), grd, blk, 0, s, static_cast<const double*>(src),
                           static_cast<double*>(dst), p, fp);
    return hipGetLastError();
}

hipError_t launch_step_eigen(StepKind kind, int Q, const void* src, void* dst, const KParams& p,
                             const FdParams& fp, double*, hipStream_t s) {
    return Q == 9 ? eig_q<9>(kind, src, dst, p, fp, s) : eig_q<19>(kind, src, dst, p, fp, s);
}

}  // namespace mlbm
