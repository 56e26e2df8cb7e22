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

// Distance of every cell from the uniform state of the global averages
// (Eqs. GlobalDensity, GlobalVelocity, GlobalTotalEnergy), which is the state
// the run converges to (Sec. 4, convergence to equilibrium), and the global
// internal and kinetic energy (Sec. 4, interference: only their sum is
// conserved).  g holds the sums of a k_moments pass already finalised:
// g[0..3] sum rho, g[4..6] sum tr rho u, g[7] sum tr rho eps_tot.
// Slots: 0 max ||rho - rho_bar|| (spectral norm), 1 max |u - u_bar|,
// 2 max |eps_tot - eps_tot_bar|, 3 sum tr rho eps, 4 sum tr rho |u|^2 / 2,
// 5..7 sums of the squares of the three distances.
template <int Q, int MODE>
__global__ void __launch_bounds__(kRedThreads)
k_relaxation(const typename Store<MODE>::T* __restrict__ W, const double* __restrict__ g, const KParams p,
             double* __restrict__ partials) {
    constexpr int D = Lat<Q>::D;
    const size_t N = static_cast<size_t>(p.ncell);
    const double invN = 1.0 / static_cast<double>(N);
    const double rho_bar[4] = {g[0] * invN, g[1] * invN, g[2] * invN, g[3] * invN};
    const double u_bar[3] = {g[4] / g[0], g[5] / g[0], g[6] / g[0]};
    const double etot_bar = g[7] / g[0];
    double acc[kRedSlots];
#pragma unroll
    for (int s = 0; s < kRedSlots; ++s) acc[s] = 0.0;
    for (size_t n = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const size_t row = n / p.nx;
        const int x = static_cast<int>(n - row * p.nx);
        double rho[4] = {0.0, 0.0, 0.0, 0.0}, J[3] = {0.0, 0.0, 0.0}, K = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double a0 = static_cast<double>(decode<MODE>(W[fidx(Q, p.nx, row, 0, i, x)], 0, i, p));
            rho[0] += a0;
#pragma unroll
            for (int c = 0; c < 3; ++c) J[c] += Lat<Q>::c(i, c) * a0;
            K += csq<Q>(i) * a0;
#pragma unroll
            for (int k = 1; k < 4; ++k) rho[k] += static_cast<double>(decode<MODE>(W[fidx(Q, p.nx, row, k, i, x)], k, i, p));
        }
        const double T = rho[0];
        double uu = 0.0, du2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double uc = (c < D) ? p.xi * J[c] / T : 0.0;
            uu += uc * uc;
            du2 += (uc - u_bar[c]) * (uc - u_bar[c]);
        }
        const double etot = p.half_xi2 * K;     // tr rho eps_tot of the cell
        // (rho - rho_bar) = (d0 I + d . sigma) / 2 has eigenvalues (d0 +- |d|) / 2
        const double d0 = rho[0] - rho_bar[0];
        const double dv = sqrt((rho[1] - rho_bar[1]) * (rho[1] - rho_bar[1]) +
                               (rho[2] - rho_bar[2]) * (rho[2] - rho_bar[2]) +
                               (rho[3] - rho_bar[3]) * (rho[3] - rho_bar[3]));
        const double drho = 0.5 * (fabs(d0) + dv);
        const double du = sqrt(du2);
        const double de = fabs(etot / T - etot_bar);
        acc[0] = fmax(acc[0], drho);
        acc[1] = fmax(acc[1], du);
        acc[2] = fmax(acc[2], de);
        acc[3] += etot - 0.5 * T * uu;
        acc[4] += 0.5 * T * uu;
        acc[5] += drho * drho;
        acc[6] += du2;
        acc[7] += de * de;
    }
    block_reduce_store<7u>(acc, partials + blockIdx.x * kRedSlots);
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
        // rows t, t + kRedThreads, ... in order; eight loads in flight at a time
        for (int j0 = t; j0 < nblocks && s < stride; j0 += 8 * kRedThreads) {
            double o[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + q * kRedThreads;
                o[q] = partials[static_cast<size_t>(j < nblocks ? j : nblocks - 1) * stride + s];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (j0 + q * kRedThreads < nblocks) v = is_max ? fmax(v, o[q]) : v + o[q];
            }
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

// First stage of a long sum: block b reduces the consecutive chunk
// [b chunk, (b + 1) chunk) of x (each thread a fixed stride, then a fixed LDS
// tree) into out[b].  Reproducible for a given n.
__global__ void __launch_bounds__(kRedThreads)
k_chunk_sums(const double* __restrict__ x, size_t n, size_t chunk, double* __restrict__ out) {
    __shared__ double sh[kRedThreads];
    const int t = threadIdx.x;
    const size_t lo = static_cast<size_t>(blockIdx.x) * chunk;
    const size_t hi = lo + chunk < n ? lo + chunk : n;
    double v = 0.0;
    for (size_t j0 = lo + t; j0 < hi; j0 += 8 * kRedThreads) {
        double o[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const size_t j = j0 + q * kRedThreads;
            o[q] = x[j < hi ? j : hi - 1];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (j0 + q * kRedThreads < hi) v += o[q];
        }
    }
    sh[t] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) out[blockIdx.x] = sh[0];
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
static hipError_t relax_q(const void* W, const double* g, const KParams& p, double* partials, hipStream_t s) {
    using T = typename Store<MODE>::T;
    hipLaunchKernelGGL((k_relaxation<Q, MODE>), dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                       static_cast<const T*>(W), g, p, partials);
    return hipGetLastError();
}

hipError_t launch_relaxation(int Q, int mode, const void* W, const double* g, const KParams& p, double* partials,
                             hipStream_t s) {
    if (Q == 9) {
        if (mode == kF64) return relax_q<9, kF64>(W, g, p, partials, s);
        if (mode == kF32) return relax_q<9, kF32>(W, g, p, partials, s);
        return relax_q<9, kF16Dev>(W, g, p, partials, s);
    }
    if (mode == kF64) return relax_q<19, kF64>(W, g, p, partials, s);
    if (mode == kF32) return relax_q<19, kF32>(W, g, p, partials, s);
    return relax_q<19, kF16Dev>(W, g, p, partials, s);
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

hipError_t launch_sum_into(const double* x, size_t n, double* tail, double* accumulate_into, double scale0,
                           hipStream_t s) {
    if (n <= static_cast<size_t>(kSumDirect))
        return launch_finalize(x, static_cast<int>(n), 1, 0u, nullptr, accumulate_into, scale0, s);
    // chunk: a multiple of the block size, so that at most kSumChunks chunks cover n
    const size_t per = (n + kSumChunks - 1) / kSumChunks;
    const size_t chunk = (per + kRedThreads - 1) / kRedThreads * kRedThreads;
    const size_t nchunk = (n + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_chunk_sums, dim3(static_cast<unsigned>(nchunk)), dim3(kRedThreads), 0, s, x, n, chunk, tail);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    return launch_finalize(tail, static_cast<int>(nchunk), 1, 0u, nullptr, accumulate_into, scale0, s);
}

hipError_t launch_finalize(const double* partials, int nblocks, int stride, unsigned max_mask, double* out,
                           double* accumulate_into, double scale0, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, s, partials, nblocks, stride, max_mask, out,
                       accumulate_into, scale0);
    return hipGetLastError();
}

}  // namespace mlbm
