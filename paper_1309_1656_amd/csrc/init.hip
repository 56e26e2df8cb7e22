// Discrete Fermi-Dirac equilibrium from per-cell macroscopic data
// (Eq. WeqDiscr with U diag(n_up, n_dn) U* = rho; Eqs. WFermiDirac,
// nFDstdOmega, energyFDstdOmega).
//
// Two ways to name the state of a cell (SRC):
//  * kFromDensity: rho = (tr rho I + r . sigma)/2 has eigenvalues
//    n_up/dn = (tr rho +- |r|)/2; each channel's nu = beta mu solves
//    n = (2 pi / beta)^(d/2) F_{d/2-1}(nu) in double;
//  * kFromChemical: nu_up/dn = beta mu_up/dn are given with a spin axis a
//    (unit vector, default z); n_up/dn follow from Eq. nFDstdOmega and
//    rho = U diag(n_up, n_dn) U* = ((n_up + n_dn) I + (n_up - n_dn) a . sigma)/2.
// Then eps is the Fermi-Dirac internal energy of the two channels and
// W_i = w_i rho P_i(u, eps).
#include "common.hpp"
#include "fermi_device.hpp"
#include "internal.hpp"
#include "reduce.hpp"

namespace mlbm {

template <int Q, int MODE, int PHASE, int SRC>
__global__ void __launch_bounds__(kRedThreads)
k_init(typename Store<MODE>::T* __restrict__ W, const double* __restrict__ rho4, const double* __restrict__ axis,
       const double* __restrict__ u_in, const double* __restrict__ T_in, const KParams p, const FdParams fp,
       double* __restrict__ partials) {
    constexpr int D = Lat<Q>::D;
    const size_t N = static_cast<size_t>(p.ncell);
    double acc[kRedSlots];
#pragma unroll
    for (int s = 0; s < kRedSlots; ++s) acc[s] = 0.0;

    for (size_t n = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<size_t>(gridDim.x) * blockDim.x) {
        double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < D; ++c) u[c] = u_in[c * N + n];
        const double T = T_in[n];
        const double beta = 1.0 / T;
        bool ok = T > 0.0 && isfinite(T) && isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]);
        double trr, r[3], nu_up, nu_dn;
        if constexpr (SRC == kFromDensity) {
            trr = rho4[n];
            r[0] = rho4[N + n];
            r[1] = rho4[2 * N + n];
            r[2] = rho4[3 * N + n];
            const double absr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            ok = ok && trr > 0.0 && absr < trr && isfinite(trr) && isfinite(absr);
            if (!ok) {
                acc[8] += 1.0;
                continue;
            }
            if (!fd::channel_nu<D>(0.5 * (trr + absr), beta, nu_up) ||
                !fd::channel_nu<D>(0.5 * (trr - absr), beta, nu_dn)) {
                acc[9] += 1.0;
                continue;
            }
        } else {
            nu_up = rho4[n];
            nu_dn = rho4[N + n];
            double a[3] = {0.0, 0.0, 1.0};
            if (axis) {
                a[0] = axis[n];
                a[1] = axis[N + n];
                a[2] = axis[2 * N + n];
            }
            const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            // the series and quadrature of F_k cover nu <= kXMax
            ok = ok && na > 0.0 && isfinite(na) && nu_up <= fd::kXMax && nu_dn <= fd::kXMax && isfinite(nu_up) &&
                 isfinite(nu_dn);
            if (!ok) {
                acc[8] += 1.0;
                continue;
            }
            const double n_up = fd::channel_density<D>(beta, nu_up), n_dn = fd::channel_density<D>(beta, nu_dn);
            trr = n_up + n_dn;
#pragma unroll
            for (int c = 0; c < 3; ++c) r[c] = (n_up - n_dn) * (a[c] / na);
        }
        const double eps = fd::internal_energy<D>(beta, nu_up, nu_dn, fp);
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        if (PHASE == 0) {
            acc[0] += trr;
            acc[1] += r[0];
            acc[2] += r[1];
            acc[3] += r[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[4 + c] += trr * u[c];
            acc[7] += trr * (eps + 0.5 * uu);
            continue;
        }
        // P_i of Eq. WeqAlgo in double
        const double b = p.beta0 * eps;
        const double al1 = p.a1_0 + p.a1_b * b, al2 = p.a2_0 + p.a2_b * b;
        const double rk[4] = {trr, r[0], r[1], r[2]};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double eu = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) eu += p.xi * Lat<Q>::c(i, c) * u[c];
            const double e2 = p.xi * p.xi * csq<Q>(i);
            const double P = al1 + al2 * p.beta0 * 0.5 * e2 + p.a3 * p.beta0 * eu +
                             p.a4 * (p.beta0 * eu) * (p.beta0 * eu) + p.a5 * p.beta0 * 0.5 * uu;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double wv = p.w[i] * rk[k] * P;
                if (PHASE == 1) {
                    acc[0] = fmax(acc[0], fabs(wv - static_cast<double>(p.ref[k][i])) / p.w[i]);
                } else {
                    W[fidx(Q, p.nx, n / p.nx, k, i, static_cast<int>(n % p.nx))] =
                        encode<MODE>(static_cast<typename Store<MODE>::C>(wv), k, i, p);
                }
            }
        }
    }
    block_reduce_store<(PHASE == 1) ? 1u : 0u>(acc, partials + blockIdx.x * kRedSlots);
}

template <int Q, int MODE, int SRC>
static hipError_t init_q(int phase, void* W, const double* a, const double* axis, const double* u, const double* T,
                         const KParams& p, const FdParams& fp, double* partials, hipStream_t s) {
    using Tp = typename Store<MODE>::T;
    Tp* w = static_cast<Tp*>(W);
    const dim3 g(kRedBlocks), b(kRedThreads);
    if (phase == 0)
        hipLaunchKernelGGL((k_init<Q, MODE, 0, SRC>), g, b, 0, s, w, a, axis, u, T, p, fp, partials);
    else if (phase == 1)
        hipLaunchKernelGGL((k_init<Q, MODE, 1, SRC>), g, b, 0, s, w, a, axis, u, T, p, fp, partials);
    else
        hipLaunchKernelGGL((k_init<Q, MODE, 2, SRC>), g, b, 0, s, w, a, axis, u, T, p, fp, partials);
    return hipGetLastError();
}

template <int SRC>
static hipError_t init_src(int Q, int mode, int phase, void* W, const double* a, const double* axis, const double* u,
                           const double* T, const KParams& p, const FdParams& fp, double* partials, hipStream_t s) {
    if (Q == 9) {
        if (mode == kF64) return init_q<9, kF64, SRC>(phase, W, a, axis, u, T, p, fp, partials, s);
        if (mode == kF32) return init_q<9, kF32, SRC>(phase, W, a, axis, u, T, p, fp, partials, s);
        return init_q<9, kF16Dev, SRC>(phase, W, a, axis, u, T, p, fp, partials, s);
    }
    if (mode == kF64) return init_q<19, kF64, SRC>(phase, W, a, axis, u, T, p, fp, partials, s);
    if (mode == kF32) return init_q<19, kF32, SRC>(phase, W, a, axis, u, T, p, fp, partials, s);
    return init_q<19, kF16Dev, SRC>(phase, W, a, axis, u, T, p, fp, partials, s);
}

hipError_t launch_init(int Q, int mode, int phase, int src, void* W, const double* a, const double* axis,
                       const double* u, const double* T, const KParams& p, const FdParams& fp, double* partials,
                       hipStream_t s) {
    if (src == kFromChemical) return init_src<kFromChemical>(Q, mode, phase, W, a, axis, u, T, p, fp, partials, s);
    return init_src<kFromDensity>(Q, mode, phase, W, a, axis, u, T, p, fp, partials, s);
}

}  // namespace mlbm
