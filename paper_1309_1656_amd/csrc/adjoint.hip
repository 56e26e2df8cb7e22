// Reverse-mode derivative of one step W_{n+1} = S(C(W_n)) (Eqs. CollisionStep,
// TransportStep), derived from Sec. 3.3.
//
// With g_i(x) = lam_{n+1,i}(x + c_i) (transpose of the streaming
// permutation), rho_k = sum_i a_ik, wP_i = w_i P_i and G_i = w_i sum_k g_ik rho_k:
//   lam_n_jk = (1 - omega) g_jk + omega sum_i wP_i g_ik
//              + [k = 0] omega (G_u . (e_j - u) + G_eps (|e_j - u|^2/2 - eps)) / T,
//   G_u  = sum_i G_i dP_i/du,   dP_i/du  = beta0 xi c_i (alpha3 + 2 alpha4 c_i.v) + alpha5 beta0 u,
//   G_eps = sum_i G_i dP_i/deps, dP_i/deps = beta0 (a1_b + a2_b beta0 xi^2 |c_i|^2 / 2),
//   dL/domega += sum_{i,k} g_ik (wP_i rho_k - a_ik),
// where v = beta0 xi u, and du/d(tr W_j) = (e_j - u)/T,
// deps/d(tr W_j) = (|e_j - u|^2/2 - eps)/T.
//
// Fields are read in the storage type.  Two organisations of the same
// arithmetic:
// * channel-parallel (k_adjoint_channel, the default without a magnetic
//   field): the step kernels' row-blocked cells with one wave per Pauli
//   channel, so that every wave streams only the Q segments of its channel of
//   each of the three fields.  The trace wave's moments reach the other waves
//   through LDS; the Bloch waves hand back their parts of G_u, sum_i G_i and
//   G_eps, which are linear in the G_i.  Per-population products are formed
//   in the compute type of the storage (float for FP32, as in the step
//   kernels) and summed in double.
// * one thread per cell with all four channels: the trace channel is handled
//   first and last so that each Bloch channel k = 1..3 is loaded, used and
//   written in turn.  The wide form (D2Q9) loads a cell's values up front and
//   holds the per-velocity factors; the staged one (D3Q19) holds one channel
//   at a time and folds G_i into G_u, sum_i G_i and G_eps as it goes.  With a
//   magnetic field (FIELD) the Bloch part of g is turned back by the transpose
//   of the cell's rotation before it enters the collision's adjoint; that
//   rotation mixes the three Bloch channels of a value, so the field runs in
//   this form only.  All its arithmetic is in double.
//
// W_n can be read as stored (WPULL = false) or gathered from the previous
// post-collision state S_{n-1}, W_n,i(x) = S_{n-1},i(x - c_i) (WPULL = true),
// so that a recomputed segment needs one fused pass per state.
#include "block_order.hpp"
#include "common.hpp"
#include "internal.hpp"

namespace mlbm {

// Periodic neighbour coordinates of a push: index [c + 1] holds (x + c) mod n.
__device__ __forceinline__ void push_coords(int x, int n, int stride, int out[3]) {
    out[0] = ((x == 0) ? n - 1 : x - 1) * stride;
    out[1] = x * stride;
    out[2] = ((x + 1 == n) ? 0 : x + 1) * stride;
}

// Empty register barriers: the compiler must assume the values changed, so it
// recomputes what depends on them instead of holding Q copies across the
// channel loop (register pressure sets the occupancy of this kernel).
__device__ __forceinline__ void opaque(double& a, double& b, double& c, double& d, double& e) {
    asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d), "+v"(e));
}
template <typename T> __device__ __forceinline__ void keep(T& a) { asm volatile("" : "+v"(a)); }
// The same for accumulated sums: their terms are computed here, not sunk to
// the (late) use together with every value they depend on.
__device__ __forceinline__ void settle(double& a, double& b, double& c, double& d, double& e, double& f,
                                       double& g) {
    asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d), "+v"(e), "+v"(f), "+v"(g));
}
__device__ __forceinline__ void opaque_coords(int (&a)[3], int (&b)[3], int (&c)[3]) {
    asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(b[0]), "+v"(b[1]), "+v"(b[2]));
    asm volatile("" : "+v"(c[0]), "+v"(c[1]), "+v"(c[2]));
}

// c_i . v with the zero components of c_i left out (c_i in {-1, 0, 1}^3).
template <int Q>
__device__ __forceinline__ double cdot(int i, const double v[3]) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (Lat<Q>::c(i, c) > 0) s += v[c];
        if (Lat<Q>::c(i, c) < 0) s -= v[c];
    }
    return s;
}

// Wide form: every value of the cell is loaded up front and the per-velocity
// factors are held in registers.  Used for D2Q9, whose 4 Q values per field
// fit in registers with three waves per SIMD.
template <int Q, int MODE, bool WPULL, int FIELD>
__global__ void __launch_bounds__(256)
k_adjoint_wide(const typename Store<MODE>::T* __restrict__ Wn, const typename Store<MODE>::T* __restrict__ ln1,
          typename Store<MODE>::T* __restrict__ ln, const KParams p, double* __restrict__ partials,
          const int accumulate) {
    using T = typename Store<MODE>::T;
    constexpr int D = Lat<Q>::D;
    __shared__ double sh[256];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double dom = 0.0;
    if (x < p.nx && y < p.ny) {
        const int nx = p.nx, ny = p.ny, nz = p.nz;
        const size_t row = static_cast<size_t>(z) * ny + y;
        // neighbour coordinates x + c along each axis, indexed by c + 1
        int xp[3], yp[3], zp[3] = {z, z, z};
        push_coords(x, nx, 1, xp);
        push_coords(y, ny, 1, yp);
        if constexpr (D == 3) push_coords(z, nz, 1, zp);
        size_t srow[Q], wrow[Q];
        int sx[Q], wx[Q];
        int xm[3], ym[3], zm[3] = {z, z, z};
        pull_coords(x, nx, 1, xm);
        pull_coords(y, ny, 1, ym);
        if constexpr (D == 3) pull_coords(z, nz, 1, zm);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            srow[i] = static_cast<size_t>(zp[Lat<Q>::c(i, 2) + 1]) * ny + yp[Lat<Q>::c(i, 1) + 1];
            sx[i] = xp[Lat<Q>::c(i, 0) + 1];
            wrow[i] = WPULL ? static_cast<size_t>(zm[Lat<Q>::c(i, 2) + 1]) * ny + ym[Lat<Q>::c(i, 1) + 1] : row;
            wx[i] = WPULL ? xm[Lat<Q>::c(i, 0) + 1] : x;
        }
        // trace channel of W_n: moments and the polynomial factor
        double a0[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) a0[i] = static_cast<double>(Wn[fidx(Q, nx, wrow[i], 0, i, wx[i])]);
        double Tr = 0.0, J[3] = {0.0, 0.0, 0.0}, K = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            Tr += a0[i];
#pragma unroll
            for (int c = 0; c < 3; ++c) J[c] += Lat<Q>::c(i, c) * a0[i];
            K += csq<Q>(i) * a0[i];
        }
        const double invT = 1.0 / Tr;
        double u[3], uu = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u[c] = (c < D) ? p.xi * J[c] * invT : 0.0;
            uu += u[c] * u[c];
        }
        const double eps = p.half_xi2 * K * invT - 0.5 * uu;
        const double b = p.beta0 * eps;
        const double A = p.a1_0 + p.a1_b * b + p.a5 * p.beta0 * 0.5 * uu;
        const double B = (p.a2_0 + p.a2_b * b) * p.beta0 * p.half_xi2;
        const double bx = p.beta0 * p.xi;
        double wP[Q], cv[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            cv[i] = bx * (Lat<Q>::c(i, 0) * u[0] + Lat<Q>::c(i, 1) * u[1] + Lat<Q>::c(i, 2) * u[2]);
            wP[i] = p.w[i] * (A + B * csq<Q>(i) + cv[i] * (p.a3 + p.a4 * cv[i]));
        }
        const double om = p.om, omm = p.one_m_om;
        // trace channel of lam_{n+1}, gathered from x + c_i
        double g0[Q], G[Q];
        double h0 = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            g0[i] = static_cast<double>(ln1[fidx(Q, nx, srow[i], 0, i, sx[i])]);
            h0 += g0[i] * wP[i];
            dom += g0[i] * (wP[i] * Tr - a0[i]);
            G[i] = p.w[i] * g0[i] * Tr;
        }
        // With a magnetic field the collision output was turned by the Bloch
        // rotation R of the cell (Sec. 5, Eq. sigmaB_comm) before streaming; its
        // adjoint turns the Bloch part of g back: g'_l = sum_k R_kl g_k.
        double gB[FIELD != kFieldNone ? 3 : 1][FIELD != kFieldNone ? Q : 1];
        if constexpr (FIELD != kFieldNone) {
            double R[9];
            if constexpr (FIELD == kFieldUniform) {
#pragma unroll
                for (int j = 0; j < 9; ++j) R[j] = p.rot[j];
            } else {
                const size_t cell = row * nx + x;
                const size_t N = static_cast<size_t>(p.ncell);
                const double bm[3] = {p.bmap[cell], p.bmap[N + cell], p.bmap[2 * N + cell]};
                rotation_matrix(bm, R);
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                double v[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) v[k] = static_cast<double>(ln1[fidx(Q, nx, srow[i], k + 1, i, sx[i])]);
#pragma unroll
                for (int l = 0; l < 3; ++l) gB[l][i] = R[l] * v[0] + R[3 + l] * v[1] + R[6 + l] * v[2];
            }
        }
        // Bloch channels
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            double ak[Q], gk[Q];
            double rk = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                ak[i] = static_cast<double>(Wn[fidx(Q, nx, wrow[i], k, i, wx[i])]);
                rk += ak[i];
            }
            double hk = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if constexpr (FIELD != kFieldNone) gk[i] = gB[k - 1][i];
                else gk[i] = static_cast<double>(ln1[fidx(Q, nx, srow[i], k, i, sx[i])]);
                hk += gk[i] * wP[i];
                dom += gk[i] * (wP[i] * rk - ak[i]);
                G[i] += p.w[i] * gk[i] * rk;
            }
            const double mix = om * hk;
#pragma unroll
            for (int i = 0; i < Q; ++i) ln[fidx(Q, nx, row, k, i, x)] = static_cast<T>(omm * gk[i] + mix);
        }
        // G_u, G_eps and the trace-channel output
        double Gu[3] = {0.0, 0.0, 0.0}, Gsum = 0.0, Ge = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double f = G[i] * bx * (p.a3 + 2.0 * p.a4 * cv[i]);
#pragma unroll
            for (int c = 0; c < 3; ++c) Gu[c] += Lat<Q>::c(i, c) * f;
            Gsum += G[i];
            Ge += G[i] * (p.a1_b + p.a2_b * p.beta0 * p.half_xi2 * csq<Q>(i));
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) Gu[c] += p.a5 * p.beta0 * u[c] * Gsum;
        Ge *= p.beta0;
        const double mix0 = om * h0;
        const double sc = om * invT;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            double gdu = 0.0, dev2 = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double dv = p.xi * Lat<Q>::c(j, c) - u[c];
                gdu += Gu[c] * dv;
                dev2 += dv * dv;
            }
            ln[fidx(Q, nx, row, 0, j, x)] = static_cast<T>(omm * g0[j] + mix0 + sc * (gdu + Ge * (0.5 * dev2 - eps)));
        }
    }
    // block partial of dL/domega (fixed tree: reproducible)
    sh[tid] = dom;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        partials[bid] = accumulate ? partials[bid] + sh[0] : sh[0];
    }
}

// Staged form: the trace channels first, then one Bloch channel at a time,
// with per-velocity factors recomputed rather than held, so that D3Q19 keeps
// two waves per SIMD (the wide form needs over 256 registers there).
template <int Q, int MODE, bool WPULL, int FIELD>
__global__ void __launch_bounds__(256)
k_adjoint_staged(const typename Store<MODE>::T* __restrict__ Wn, const typename Store<MODE>::T* __restrict__ ln1,
          typename Store<MODE>::T* __restrict__ ln, const KParams p, double* __restrict__ partials,
          const int accumulate) {
    using T = typename Store<MODE>::T;
    constexpr int D = Lat<Q>::D;
    __shared__ double sh[256];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double dom = 0.0;
    if (x < p.nx && y < p.ny) {
        const int nx = p.nx, ny = p.ny, nz = p.nz;
        const size_t row = static_cast<size_t>(z) * ny + y;
        const size_t seg = static_cast<size_t>(Q) * nx;      // one Pauli component of a row
        // neighbour coordinates x + c (lam gather) and x - c (W pull), indexed by c + 1
        int xp[3], yp[3], zp[3] = {z, z, z};
        push_coords(x, nx, 1, xp);
        push_coords(y, ny, 1, yp);
        if constexpr (D == 3) push_coords(z, nz, 1, zp);
        int xm[3], ym[3], zm[3] = {z, z, z};
        if constexpr (WPULL) {
            pull_coords(x, nx, 1, xm);
            pull_coords(y, ny, 1, ym);
            if constexpr (D == 3) pull_coords(z, nz, 1, zm);
        }
        // element offset of (Pauli component 0, velocity i) at the lam and W gather positions
        auto lam_at = [&](int i) -> size_t {
            const size_t r = static_cast<size_t>(zp[Lat<Q>::c(i, 2) + 1]) * ny + yp[Lat<Q>::c(i, 1) + 1];
            return r * 4 * seg + static_cast<size_t>(i) * nx + xp[Lat<Q>::c(i, 0) + 1];
        };
        auto w_at = [&](int i) -> size_t {
            if constexpr (WPULL) {
                const size_t r = static_cast<size_t>(zm[Lat<Q>::c(i, 2) + 1]) * ny + ym[Lat<Q>::c(i, 1) + 1];
                return r * 4 * seg + static_cast<size_t>(i) * nx + xm[Lat<Q>::c(i, 0) + 1];
            } else {
                return row * 4 * seg + static_cast<size_t>(i) * nx + x;
            }
        };
        const size_t own = row * 4 * seg + x;      // + (k Q + i) nx

        // trace channels: moments of W_n and the polynomial factor
        T a0[Q], g0[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            a0[i] = Wn[w_at(i)];
            g0[i] = ln1[lam_at(i)];
        }
        double Tr = 0.0, J[3] = {0.0, 0.0, 0.0}, K = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double a = static_cast<double>(a0[i]);
            Tr += a;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (Lat<Q>::c(i, c) > 0) J[c] += a;
                if (Lat<Q>::c(i, c) < 0) J[c] -= a;
            }
            if (csq<Q>(i) == 1) K += a;
            if (csq<Q>(i) == 2) K += 2.0 * a;
        }
        const double invT = 1.0 / Tr;
        double u[3], uu = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u[c] = (c < D) ? p.xi * J[c] * invT : 0.0;
            uu += u[c] * u[c];
        }
        const double eps = p.half_xi2 * K * invT - 0.5 * uu;
        const double b = p.beta0 * eps;
        double A = p.a1_0 + p.a1_b * b + p.a5 * p.beta0 * 0.5 * uu;
        double B = (p.a2_0 + p.a2_b * b) * p.beta0 * p.half_xi2;
        const double bx = p.beta0 * p.xi;
        // beta0 xi c_i . u and w_i P_i, recomputed where needed rather than held
        auto cv_of = [&](int i) -> double { return bx * cdot<Q>(i, u); };
        auto wP_of = [&](int i) -> double {
            const double cv = cv_of(i);
            return p.w[i] * (A + B * csq<Q>(i) + cv * (p.a3 + p.a4 * cv));
        };
        // G_i = w_i sum_k g_ik rho_k enters only through the linear forms
        // G_u = sum_i G_i dP_i/du (with the alpha5 term added at the end),
        // sum_i G_i and G_eps = sum_i G_i dP_i/deps / beta0: accumulate those.
        double Gu[3] = {0.0, 0.0, 0.0}, Gsum = 0.0, Ge = 0.0;
        auto add_G = [&](int i, double Gi) {
            const double f = Gi * bx * (p.a3 + 2.0 * p.a4 * cv_of(i));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (Lat<Q>::c(i, c) > 0) Gu[c] += f;
                if (Lat<Q>::c(i, c) < 0) Gu[c] -= f;
            }
            Gsum += Gi;
            Ge += Gi * (p.a1_b + p.a2_b * p.beta0 * p.half_xi2 * csq<Q>(i));
        };
        const double om = p.om, omm = p.one_m_om;
        double h0 = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double g = static_cast<double>(g0[i]);
            const double wP = wP_of(i);
            h0 += g * wP;
            dom += g * (wP * Tr - static_cast<double>(a0[i]));
            add_G(i, p.w[i] * g * Tr);
        }
        settle(h0, dom, Gu[0], Gu[1], Gu[2], Gsum, Ge);
        // With a magnetic field the collision output was turned by the Bloch
        // rotation R of the cell (Sec. 5, Eq. sigmaB_comm) before streaming; its
        // adjoint turns the Bloch part of g back: g'_l = sum_k R_kl g_k.
        double gB[FIELD != kFieldNone ? 3 : 1][FIELD != kFieldNone ? Q : 1];
        if constexpr (FIELD != kFieldNone) {
            double R[9];
            if constexpr (FIELD == kFieldUniform) {
#pragma unroll
                for (int j = 0; j < 9; ++j) R[j] = p.rot[j];
            } else {
                const size_t cell = row * nx + x;
                const size_t N = static_cast<size_t>(p.ncell);
                const double bm[3] = {p.bmap[cell], p.bmap[N + cell], p.bmap[2 * N + cell]};
                rotation_matrix(bm, R);
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                double v[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) v[k] = static_cast<double>(ln1[lam_at(i) + (k + 1) * seg]);
#pragma unroll
                for (int l = 0; l < 3; ++l) gB[l][i] = R[l] * v[0] + R[3 + l] * v[1] + R[6 + l] * v[2];
            }
        }
        // Bloch channels, one at a time: rho_k first, then g_k
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            // keep the scheduler from hoisting this channel's loads above the
            // previous channel's work: one channel's values in registers at a time
            __builtin_amdgcn_sched_barrier(0);
            opaque(u[0], u[1], u[2], A, B);
            opaque_coords(xp, yp, zp);
            if constexpr (WPULL) opaque_coords(xm, ym, zm);
            T ak[Q], gk[Q];
            double rk = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                ak[i] = Wn[w_at(i) + k * seg];
                if constexpr (FIELD == kFieldNone) gk[i] = ln1[lam_at(i) + k * seg];
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) rk += static_cast<double>(ak[i]);
            double hk = 0.0;
            double gd[FIELD != kFieldNone ? Q : 1];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                double g;
                if constexpr (FIELD != kFieldNone) g = gB[k - 1][i];
                else g = static_cast<double>(gk[i]);
                const double wP = wP_of(i);
                hk += g * wP;
                dom += g * (wP * rk - static_cast<double>(ak[i]));
                add_G(i, p.w[i] * g * rk);
                if constexpr (FIELD != kFieldNone) gd[i] = g;
            }
            settle(hk, dom, Gu[0], Gu[1], Gu[2], Gsum, Ge);
            const double mix = om * hk;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                double g;
                if constexpr (FIELD != kFieldNone) g = gd[i];
                else g = static_cast<double>(gk[i]);
                __builtin_nontemporal_store(static_cast<T>(omm * g + mix), ln + own + (k * Q + i) * static_cast<size_t>(nx));
            }
        }
        // trace-channel output (g0 re-read from its storage-type registers)
#pragma unroll
        for (int i = 0; i < Q; ++i) keep(g0[i]);
#pragma unroll
        for (int c = 0; c < 3; ++c) Gu[c] += p.a5 * p.beta0 * u[c] * Gsum;
        Ge *= p.beta0;
        const double mix0 = om * h0;
        const double sc = om * invT;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            double gdu = 0.0, dev2 = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double dv = p.xi * Lat<Q>::c(j, c) - u[c];
                gdu += Gu[c] * dv;
                dev2 += dv * dv;
            }
            __builtin_nontemporal_store(
                static_cast<T>(omm * static_cast<double>(g0[j]) + mix0 + sc * (gdu + Ge * (0.5 * dev2 - eps))),
                ln + own + static_cast<size_t>(j) * nx);
        }
    }
    // block partial of dL/domega (fixed tree: reproducible)
    sh[tid] = dom;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        partials[bid] = accumulate ? partials[bid] + sh[0] : sh[0];
    }
}

// Channel-parallel form: a workgroup covers BX consecutive cells of one row
// (block_order), four waves per 64 cells, wave group k owning Pauli channel k.
// Every wave gathers its channel of W_n (at x, or pulled from x - c_i) and of
// lam_{n+1} (from x + c_i) and writes its channel of lam_n; with NTS (fields
// larger than the last-level cache) the loads stream as well as the stores.
//
// Everything the collision's adjoint needs from a channel's g_i enters through
// a few moments: with P_i = A + B |c_i|^2 + (c_i.v)(alpha3 + alpha4 c_i.v)
// (v = beta0 xi u, A and B the cell's coefficient sums),
//   h_k = sum_i w_i P_i g_i = A m0 + B mc + alpha3 v.m1 + alpha4 v.M2 v,
//   G_u part  = rho_k beta0 xi (alpha3 m1 + 2 alpha4 M2 v),
//   sum_i G_i part = rho_k m0,   G_eps part = rho_k (a1_b m0 + a2_b beta0 xi^2/2 mc),
// with m0 = sum_i w_i g_i, mc = sum_i w_i |c_i|^2 g_i, m1 = sum_i w_i c_i g_i,
// M2 = sum_i w_i c_i c_i^T g_i.  Since c_i is in {-1, 0, 1}^3 these are sums of
// g_i with signs, weighted per weight class: additions only.  The trace wave
// hands v, A, B to the other waves (first barrier); every wave forms its
// moments and h_k and writes its Bloch channel at once; the Bloch waves hand
// their G parts to the trace wave (second barrier), which writes the trace
// channel.  Each wave's part of dL/domega, rho_k h_k - sum_i g_i a_i, is
// summed with the others of the block after the second barrier (one partial
// per block).
template <int Q> struct GMoments {
    static constexpr int D = Lat<Q>::D;
    static constexpr int kM2 = D == 3 ? 6 : 3;                 // entries of M2: xx, yy, (zz,) xy, (xz, yz)
};

template <int Q>
__device__ __forceinline__ void m2_index(int n, int& a, int& b) {
    if constexpr (Lat<Q>::D == 3) {
        constexpr int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
        a = ia[n];
        b = ib[n];
    } else {
        constexpr int ia[3] = {0, 1, 0}, ib[3] = {0, 1, 1};
        a = ia[n];
        b = ib[n];
    }
}

template <int Q, int MODE, bool WPULL, int BX, bool NTS>
__global__ void __launch_bounds__(BX * 4)
k_adjoint_channel(const typename Store<MODE>::T* __restrict__ Wn, const typename Store<MODE>::T* __restrict__ ln1,
                  typename Store<MODE>::T* __restrict__ ln, const KParams p, double* __restrict__ partials,
                  const int accumulate, const int order) {
    using T = typename Store<MODE>::T;
    using GM = GMoments<Q>;
    constexpr int D = Lat<Q>::D;
    constexpr int kWaves = BX / 64;           // waves per channel
    constexpr int kM2 = GM::kM2;
    static_assert(BX % 64 == 0, "a wave must not straddle two channels");
    const int lx = threadIdx.x;
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.y);   // Pauli channel, uniform per wave
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    int chunk, y, z;
    block_order(order, nx, ny, BX, chunk, y, z);
    const int x = chunk * BX + lx;
    const bool active = x < nx;
    const int xx = active ? x : nx - 1;
    const size_t row = static_cast<size_t>(z) * ny + y;
    // coordinate x + c along each axis, indexed by c + 1 (x - c is the same table reversed)
    const int xp[3] = {xx == 0 ? nx - 1 : xx - 1, xx, xx + 1 == nx ? 0 : xx + 1};
    const int yp[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0 : y + 1};
    int zp[3] = {z, z, z};
    if constexpr (D == 3) {
        zp[0] = z == 0 ? nz - 1 : z - 1;
        zp[2] = z + 1 == nz ? 0 : z + 1;
    }

    T wr[Q], gr[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
        size_t wrow = row;
        int wx = xx;
        if constexpr (WPULL) {
            wrow = static_cast<size_t>(zp[1 - cz]) * ny + yp[1 - cy];
            wx = xp[1 - cx];
        }
        const size_t lrow = static_cast<size_t>(zp[1 + cz]) * ny + yp[1 + cy];
        wr[i] = load_row<NTS>(Wn + fidx(Q, nx, wrow, k, i, 0), wx);
        gr[i] = load_row<NTS>(ln1 + fidx(Q, nx, lrow, k, i, 0), xp[1 + cx]);
    }

    // Sums start at -0.0, the exact additive identity (x + -0.0 == x for every x,
    // +0.0 included), so the compiler may drop their first addition.
    double rk = -0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) rk += static_cast<double>(wr[i]);

    // the trace wave: moments of W_n (Eq. DiscrAvr) and the coefficient sums of P_i
    // (Eq. WeqAlgo, Appendix), handed to the other waves
    constexpr int kT = 2 + D;                      // v (D components), A, B
    __shared__ double csh[kT][BX];
    __shared__ double gsh[3][2 + D][BX];           // Bloch waves: parts of G_u (D), sum_i G_i, sum_i |c_i|^2 G_i
    double u[3] = {0.0, 0.0, 0.0}, uu = 0.0, eps = 0.0, invT = 0.0;
    const double bx = p.beta0 * p.xi;
    if (k == 0) {
        double J[3] = {-0.0, -0.0, -0.0}, K = -0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double a = static_cast<double>(wr[i]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (Lat<Q>::c(i, c) > 0) J[c] += a;
                if (Lat<Q>::c(i, c) < 0) J[c] -= a;
            }
            if (csq<Q>(i) == 1) K += a;
            if (csq<Q>(i) == 2) K += 2.0 * a;
        }
        invT = 1.0 / rk;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            u[c] = p.xi * J[c] * invT;
            uu += u[c] * u[c];
        }
        eps = p.half_xi2 * K * invT - 0.5 * uu;
        const double b = p.beta0 * eps;
#pragma unroll
        for (int c = 0; c < D; ++c) csh[c][lx] = bx * u[c];
        csh[D][lx] = p.a1_0 + p.a1_b * b + p.a5 * p.beta0 * 0.5 * uu;
        csh[D + 1][lx] = (p.a2_0 + p.a2_b * b) * p.beta0 * p.half_xi2;
    }
    __syncthreads();
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = csh[c][lx];
    const double A = csh[D][lx], B = csh[D + 1][lx];

    // moments of this channel's g and sum_i g_i a_i
    double ga = -0.0, s0 = -0.0, sa = -0.0, sd = -0.0;             // g summed per weight class
    double m1a[3] = {-0.0, -0.0, -0.0}, m1d[3] = {-0.0, -0.0, -0.0};  // sum c_i g_i per class
    double m2a[3] = {-0.0, -0.0, -0.0}, m2d[kM2];                  // sum c_ia c_ib g_i per class
#pragma unroll
    for (int n = 0; n < kM2; ++n) m2d[n] = -0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double g = static_cast<double>(gr[i]);
        ga += g * static_cast<double>(wr[i]);
        if (csq<Q>(i) == 0) s0 += g;
        if (csq<Q>(i) == 1) sa += g;
        if (csq<Q>(i) == 2) sd += g;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double& m = csq<Q>(i) == 1 ? m1a[c] : m1d[c];
            if (Lat<Q>::c(i, c) > 0) m += g;
            if (Lat<Q>::c(i, c) < 0) m -= g;
        }
#pragma unroll
        for (int n = 0; n < kM2; ++n) {
            int ca, cb;
            m2_index<Q>(n, ca, cb);
            const int sgn = Lat<Q>::c(i, ca) * Lat<Q>::c(i, cb);
            if (sgn == 0) continue;
            if (csq<Q>(i) == 1) {          // an axis velocity has one nonzero component: diagonal entries only
                if (n < D) m2a[n] += g;
            } else {
                if (sgn > 0) m2d[n] += g;
                else m2d[n] -= g;
            }
        }
    }
    // weight classes: rest w[0], axis w[1], diagonal w[2 D + 1]
    const double w0 = p.w[0], wa = p.w[1], wd = p.w[2 * D + 1];
    const double m0 = w0 * s0 + wa * sa + wd * sd;
    const double mc = wa * sa + 2.0 * wd * sd;
    double m1[3] = {0.0, 0.0, 0.0}, M2v[3] = {-0.0, -0.0, -0.0}, vM2v = -0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) m1[c] = wa * m1a[c] + wd * m1d[c];
#pragma unroll
    for (int n = 0; n < kM2; ++n) {
        int ca, cb;
        m2_index<Q>(n, ca, cb);
        const double M = (n < D ? wa * m2a[n] : 0.0) + wd * m2d[n];
        M2v[ca] += M * v[cb];
        if (ca != cb) M2v[cb] += M * v[ca];
    }
    double vm1 = -0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        vm1 += v[c] * m1[c];
        vM2v += v[c] * M2v[c];
    }
    const double h = A * m0 + B * mc + p.a3 * vm1 + p.a4 * vM2v;      // sum_i w_i P_i g_i
    double dom = rk * h - ga;                                         // sum_i g_i (w_i P_i rho_k - a_i)
    // this channel's parts of G_u / (beta0 xi) (without the alpha5 term), sum_i G_i, sum_i |c_i|^2 G_i
    double Gu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < D; ++c) Gu[c] = rk * (p.a3 * m1[c] + 2.0 * p.a4 * M2v[c]);
    double Gs = rk * m0, Gc = rk * mc;
    // this wave's part of dL/domega, summed in a fixed butterfly order (reproducible)
    __shared__ double dsum[4 * kWaves];
    if (!active) dom = 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dom += __shfl_xor(dom, off, 64);
    if ((lx & 63) == 0) dsum[k * kWaves + lx / 64] = dom;
    const double om = p.om, omm = p.one_m_om;
    if (k > 0) {
        const double mix = om * h;
        if (active) {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                store_row<NTS>(static_cast<T>(omm * static_cast<double>(gr[i]) + mix), ln + fidx(Q, nx, row, k, i, 0), x);
        }
#pragma unroll
        for (int c = 0; c < D; ++c) gsh[k - 1][c][lx] = Gu[c];
        gsh[k - 1][D][lx] = Gs;
        gsh[k - 1][D + 1][lx] = Gc;
    }
    __syncthreads();
    if (k == 0) {
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
#pragma unroll
            for (int c = 0; c < D; ++c) Gu[c] += gsh[kk][c][lx];
            Gs += gsh[kk][D][lx];
            Gc += gsh[kk][D + 1][lx];
        }
        const double Ge = p.beta0 * (p.a1_b * Gs + p.a2_b * p.beta0 * p.half_xi2 * Gc);
#pragma unroll
        for (int c = 0; c < D; ++c) Gu[c] = bx * Gu[c] + p.a5 * p.beta0 * u[c] * Gs;
        // lam_n,j0 = (1 - omega) g_j + omega h_0 + omega/T (G_u.(e_j - u) + G_eps (|e_j - u|^2/2 - eps))
        //          = (1 - omega) g_j + K0 + K1.c_j + K2 |c_j|^2
        const double sc = om * invT;
        double Gu_u = -0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) Gu_u += Gu[c] * u[c];
        const double K0 = om * h + sc * (Ge * (0.5 * uu - eps) - Gu_u);
        double K1[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < D; ++c) K1[c] = sc * p.xi * (Gu[c] - Ge * u[c]);
        const double K2 = sc * Ge * p.half_xi2;
        if (active) {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                double t = K0 + (csq<Q>(j) == 1 ? K2 : (csq<Q>(j) == 2 ? 2.0 * K2 : 0.0));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (Lat<Q>::c(j, c) > 0) t += K1[c];
                    if (Lat<Q>::c(j, c) < 0) t -= K1[c];
                }
                store_row<NTS>(static_cast<T>(omm * static_cast<double>(gr[j]) + t), ln + fidx(Q, nx, row, 0, j, 0), x);
            }
        }
    }
    if (k == 0 && lx == 0) {
        double t = -0.0;
#pragma unroll
        for (int j = 0; j < 4 * kWaves; ++j) t += dsum[j];
        partials[blockIdx.x] = accumulate ? partials[blockIdx.x] + t : t;
    }
}

static dim3 adj_block(int nx) {
    int bx = nx >= 256 ? 256 : (nx >= 128 ? 128 : 64);
    return dim3(bx, 256 / bx, 1);
}

// Automatic launch shape of the adjoint, from sweeps of the kernel alone on
// MI355X (one adjoint step, D3Q19 128^3 and D2Q9 512^2): the channel form
// without a magnetic field (cell form: D3Q19 F64 710, F32 346 us; D2Q9 F64
// 35.7, F32 20.7 us), the step kernels' store rule;
//   D3Q19: 8-row interleave; FP64 64-cell blocks, at most 2 workgroups per CU
//          (635 us; 128-cell blocks 654 us), FP32 128-cell blocks uncapped
//          (307 us; 64-cell blocks 312 us); from 2^24 cells one row range per
//          XCD instead (384^3: FP64 17.42 against 17.86 ms, FP32 8.56 against
//          8.83 ms);
//   D2Q9: 64-cell blocks, uncapped; 8-row interleave, which is faster on states
//         that come from HBM as in a checkpointed reverse sweep (512^2 F32 22.5
//         against 23.7 us per step, 1024^2 F32 84 against 91 us, F64 162 against
//         168 us; a 512^2 F32 rollout of 200 steps 9.60 against 9.81 ms), except
//         F64 below 2^20 cells, one row range per XCD (512^2 sweep 41.4 against
//         42.4 us per step).
AdjointCfg adjoint_launch(int nx, int ny, int nz, int Q, int mode, int field_mode, AdjointCfg want) {
    AdjointCfg c = want;
    if (field_mode != kFieldNone) c.form = kAdjCell;
    if (c.form == kAdjAuto) c.form = kAdjChannel;
    const double cells = static_cast<double>(nx) * ny * nz;
    if (c.lc.stores < 0) {
        const double field_bytes = 4.0 * Q * cells * (mode == kF64 ? 8 : 4);
        c.lc.stores = field_bytes <= 192.0 * 1048576.0 ? 1 : 0;
    }
    if (c.lc.bx == 0) c.lc.bx = (Q == 19 && mode == kF32) ? 128 : 64;
    const bool big3d = Q == 19 && cells >= 16777216.0 && nx > 64;
    const bool small_f64_2d = Q == 9 && mode == kF64 && cells < 1048576.0;
    if (c.lc.order < 0) c.lc.order = (small_f64_2d || big3d) ? kOrderXcdRange : kOrderInterleave8;
    if (c.lc.cap < 0) c.lc.cap = (Q == 19 && mode == kF64) ? 2 : 0;
    return c;
}

int adjoint_blocks(const KParams& p, int mode, AdjointCfg want) {
    const AdjointCfg c = adjoint_launch(p.nx, p.ny, p.nz, p.Q, mode, p.field_mode, want);
    if (c.form == kAdjChannel) return ((p.nx + c.lc.bx - 1) / c.lc.bx) * p.ny * p.nz;
    const dim3 blk = adj_block(p.nx);
    return ((p.nx + blk.x - 1) / blk.x) * ((p.ny + blk.y - 1) / blk.y) * p.nz;
}

template <int Q, int MODE, bool WPULL, int BX>
static hipError_t adj_channel(const void* Wn, const void* l1, void* l0, const KParams& p, double* partials,
                              bool accumulate, const LaunchCfg& c, hipStream_t s) {
    using T = typename Store<MODE>::T;
    const auto fn = c.stores == 1 ? k_adjoint_channel<Q, MODE, WPULL, BX, false>
                                  : k_adjoint_channel<Q, MODE, WPULL, BX, true>;
    const dim3 grd(static_cast<unsigned>((p.nx + BX - 1) / BX) * p.ny * p.nz);
    const size_t dyn = lds_for_cap(reinterpret_cast<const void*>(fn), BX * 4, c.cap);
    hipLaunchKernelGGL(fn, grd, dim3(BX, 4), dyn, s, static_cast<const T*>(Wn), static_cast<const T*>(l1),
                       static_cast<T*>(l0), p, partials, accumulate ? 1 : 0, c.order);
    return hipGetLastError();
}

template <int Q, int MODE, int FIELD>
static hipError_t adj_cell(bool wpull, const void* Wn, const void* l1, void* l0, const KParams& p, double* partials,
                           bool accumulate, hipStream_t s) {
    using T = typename Store<MODE>::T;
    dim3 blk = adj_block(p.nx);
    dim3 grd((p.nx + blk.x - 1) / blk.x, (p.ny + blk.y - 1) / blk.y, p.nz);
    // measured on MI355X: the wide form is faster for D2Q9 (512^2 FP64 37.7 against
    // 42.1 us per pulled step), the staged form for D3Q19 (128^3 FP32 329 against 521 us)
    auto pick = [&]() {
        if constexpr (Q == 9) return wpull ? k_adjoint_wide<Q, MODE, true, FIELD> : k_adjoint_wide<Q, MODE, false, FIELD>;
        else return wpull ? k_adjoint_staged<Q, MODE, true, FIELD> : k_adjoint_staged<Q, MODE, false, FIELD>;
    };
    hipLaunchKernelGGL(pick(), grd, blk, 0, s, static_cast<const T*>(Wn), static_cast<const T*>(l1), static_cast<T*>(l0),
                       p, partials, accumulate ? 1 : 0);
    return hipGetLastError();
}

template <int Q, int MODE>
static hipError_t adj_q(bool wpull, const void* Wn, const void* l1, void* l0, const KParams& p, double* partials,
                        bool accumulate, AdjointCfg want, hipStream_t s) {
    const AdjointCfg c = adjoint_launch(p.nx, p.ny, p.nz, Q, MODE, p.field_mode, want);
    if (c.form == kAdjChannel) {
        if (c.lc.bx == 128) {
            return wpull ? adj_channel<Q, MODE, true, 128>(Wn, l1, l0, p, partials, accumulate, c.lc, s)
                         : adj_channel<Q, MODE, false, 128>(Wn, l1, l0, p, partials, accumulate, c.lc, s);
        }
        return wpull ? adj_channel<Q, MODE, true, 64>(Wn, l1, l0, p, partials, accumulate, c.lc, s)
                     : adj_channel<Q, MODE, false, 64>(Wn, l1, l0, p, partials, accumulate, c.lc, s);
    }
    if (p.field_mode == kFieldUniform) return adj_cell<Q, MODE, kFieldUniform>(wpull, Wn, l1, l0, p, partials, accumulate, s);
    if (p.field_mode == kFieldMap) return adj_cell<Q, MODE, kFieldMap>(wpull, Wn, l1, l0, p, partials, accumulate, s);
    return adj_cell<Q, MODE, kFieldNone>(wpull, Wn, l1, l0, p, partials, accumulate, s);
}

hipError_t launch_adjoint(int Q, int mode, bool wpull, const void* Wn, const void* lam_next, void* lam_n,
                          const KParams& p, double* partials, bool accumulate, AdjointCfg want, hipStream_t s) {
    if (Q == 9) return mode == kF64 ? adj_q<9, kF64>(wpull, Wn, lam_next, lam_n, p, partials, accumulate, want, s)
                                    : adj_q<9, kF32>(wpull, Wn, lam_next, lam_n, p, partials, accumulate, want, s);
    return mode == kF64 ? adj_q<19, kF64>(wpull, Wn, lam_next, lam_n, p, partials, accumulate, want, s)
                        : adj_q<19, kF32>(wpull, Wn, lam_next, lam_n, p, partials, accumulate, want, s);
}

}  // namespace mlbm
