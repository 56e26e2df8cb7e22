// Per-cell moments (Eq. DiscrAvr), global conserved averages
// (Eqs. GlobalDensity, GlobalVelocity, GlobalTotalEnergy), diagnostics, the
// final spin-density loss and the fixed-order finalisation of block partials.
#include "common.hpp"
#include "internal.hpp"
#include "reduce.hpp"

namespace mlbm {

// Grid-stride over cells; kRedBlocks x kRedThreads threads.
template <int Q, int MODE>
__global__ void __launch_bounds__(kRedThreads)
k_moments(const typename Store<MODE>::T* __restrict__ W, double* __restrict__ rho4, double* __restrict__ u_out,
          double* __restrict__ eps_out, const KParams p, double* __restrict__ partials) {
    constexpr int D = Lat<Q>::D;
    const size_t N = static_cast<size_t>(p.ncell);
    double acc[kRedSlots];
#pragma unroll
    for (int s = 0; s < kRedSlots; ++s) acc[s] = 0.0;

    for (size_t n = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const size_t row = n / p.nx;
        const int x = static_cast<int>(n - row * p.nx);
        double a[4][Q];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int i = 0; i < Q; ++i)
                a[k][i] = static_cast<double>(decode<MODE>(W[fidx(Q, p.nx, row, k, i, x)], k, i, p));
        double rho[4] = {0.0, 0.0, 0.0, 0.0}, J[3] = {0.0, 0.0, 0.0}, K = 0.0;
        double nneg = 0.0, nbad = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                rho[k] += a[k][i];
                if (!isfinite(a[k][i])) nbad += 1.0;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) J[c] += Lat<Q>::c(i, c) * a[0][i];
            K += csq<Q>(i) * a[0][i];
            // eigenvalues (a0 +- |a|)/2 of the population
            const double m = sqrt(a[1][i] * a[1][i] + a[2][i] * a[2][i] + a[3][i] * a[3][i]);
            if (a[0][i] - m < 0.0) nneg += 1.0;
        }
        const double T = rho[0];
        double uu = 0.0, uv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uv[c] = (c < D) ? p.xi * J[c] / T : 0.0;
            uu += uv[c] * uv[c];
        }
        const double etot = p.half_xi2 * K;         // sum_i |e_i|^2 / 2 tr W_i
        if (rho4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) rho4[k * N + n] = rho[k];
        }
        if (u_out) {
#pragma unroll
            for (int c = 0; c < D; ++c) u_out[c * N + n] = uv[c];
        }
        if (eps_out) eps_out[n] = etot / T - 0.5 * uu;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += rho[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[4 + c] += (c < D) ? p.xi * J[c] : 0.0;
        acc[7] += etot;
        acc[8] += nneg;
        acc[9] += nbad;
    }
    block_reduce_store<0u>(acc, partials + blockIdx.x * kRedSlots);
}

template <int Q, int MODE>
__global__ void __launch_bounds__(kRedThreads)
k_spin_loss(const typename Store<MODE>::T* __restrict__ W, const double* __restrict__ rt,
            typename Store<MODE>::T* __restrict__ lam, const KParams p, double* __restrict__ partials) {
    using T = typename Store<MODE>::T;
    const size_t N = static_cast<size_t>(p.ncell);
    const double g = 2.0 / static_cast<double>(N);
    double acc[kRedSlots];
#pragma unroll
    for (int s = 0; s < kRedSlots; ++s) acc[s] = 0.0;
    for (size_t n = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const size_t row = n / p.nx;
        const int x = static_cast<int>(n - row * p.nx);
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            double r = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) r += static_cast<double>(W[fidx(Q, p.nx, row, k, i, x)]);
            const double diff = r - rt[(k - 1) * N + n];
            acc[0] += diff * diff;
            if (lam) {
                const T s = static_cast<T>(g * diff);
#pragma unroll
                for (int i = 0; i < Q; ++i) lam[fidx(Q, p.nx, row, k, i, x)] = s;
            }
        }
        if (lam) {
#pragma unroll
            for (int i = 0; i < Q; ++i) lam[fidx(Q, p.nx, row, 0, i, x)] = T(0);
        }
    }
    block_reduce_store<0u>(acc, partials + blockIdx.x * kRedSlots);
}

__global__ void __launch_bounds__(kRedThreads)
k_finalize(const double* __restrict__ partials, int nblocks, int stride, unsigned max_mask,
           double* __restrict__ out, double* __restrict__ accumulate_into, double scale0) {
    __shared__ double sh[kRedSlots][kRedThreads];
    const int t = threadIdx.x;
    for (int s = 0; s < kRedSlots; ++s) {
        const bool is_max = (max_mask >> s) & 1u;
        double v = is_max ? -1.0e300 : 0.0;
        for (int j = t; j < nblocks && s < stride; j += kRedThreads) {
            const double o = partials[static_cast<size_t>(j) * stride + s];
            v = is_max ? fmax(v, o) : v + o;
        }
        sh[s][t] = v;
    }
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            for (int s = 0; s < kRedSlots; ++s) {
                const double o = sh[s][t + w];
                sh[s][t] = ((max_mask >> s) & 1u) ? fmax(sh[s][t], o) : sh[s][t] + o;
            }
        }
        __syncthreads();
    }
    if (t < kRedSlots) {
        if (accumulate_into) {
            if (t == 0) accumulate_into[0] += scale0 * sh[0][0];
        } else {
            out[t] = (t == 0) ? scale0 * sh[0][0] : sh[t][0];
        }
    }
}

template <int Q, int MODE>
static hipError_t moments_q(const void* W, double* rho4, double* u, double* eps, const KParams& p,
                            double* partials, hipStream_t s) {
    using T = typename Store<MODE>::T;
    hipLaunchKernelGGL((k_moments<Q, MODE>), dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                       static_cast<const T*>(W), rho4, u, eps, p, partials);
    return hipGetLastError();
}

hipError_t launch_moments(int Q, int mode, const void* W, double* rho4, double* u, double* eps,
                          const KParams& p, double* partials, hipStream_t s) {
    if (Q == 9) {
        if (mode == kF64) return moments_q<9, kF64>(W, rho4, u, eps, p, partials, s);
        if (mode == kF32) return moments_q<9, kF32>(W, rho4, u, eps, p, partials, s);
        return moments_q<9, kF16Dev>(W, rho4, u, eps, p, partials, s);
    }
    if (mode == kF64) return moments_q<19, kF64>(W, rho4, u, eps, p, partials, s);
    if (mode == kF32) return moments_q<19, kF32>(W, rho4, u, eps, p, partials, s);
    return moments_q<19, kF16Dev>(W, rho4, u, eps, p, partials, s);
}

template <int Q, int MODE>
static hipError_t loss_q(const void* W, const double* rt, void* lam, const KParams& p, double* partials,
                         hipStream_t s) {
    using T = typename Store<MODE>::T;
    hipLaunchKernelGGL((k_spin_loss<Q, MODE>), dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                       static_cast<const T*>(W), rt, static_cast<T*>(lam), p, partials);
    return hipGetLastError();
}

hipError_t launch_spin_loss(int Q, int mode, const void* W, const double* r_target, void* lam,
                            const KParams& p, double* partials, hipStream_t s) {
    if (Q == 9) return mode == kF64 ? loss_q<9, kF64>(W, r_target, lam, p, partials, s)
                                    : loss_q<9, kF32>(W, r_target, lam, p, partials, s);
    return mode == kF64 ? loss_q<19, kF64>(W, r_target, lam, p, partials, s)
                        : loss_q<19, kF32>(W, r_target, lam, p, partials, s);
}

hipError_t launch_finalize(const double* partials, int nblocks, int stride, unsigned max_mask, double* out,
                           double* accumulate_into, double scale0, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, s, partials, nblocks, stride, max_mask, out,
                       accumulate_into, scale0);
    return hipGetLastError();
}

}  // namespace mlbm
