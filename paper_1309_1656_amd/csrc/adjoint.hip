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
// One thread per cell; fields are read in the storage type and all
// arithmetic is in double.  The trace channel is handled first and last so
// that each Bloch channel k = 1..3 is loaded, used and written in turn.  Two
// forms of the same arithmetic: the wide one (D2Q9) loads a cell's values up
// front and holds the per-velocity factors; the staged one (D3Q19) holds one
// channel at a time and folds G_i into G_u, sum_i G_i and G_eps as it goes,
// which halves its registers and doubles the waves per SIMD.
//
// With a magnetic field (FIELD) the Bloch part of g is turned back by the
// transpose of the cell's rotation before it enters the collision's adjoint.
//
// W_n can be read as stored (WPULL = false) or gathered from the previous
// post-collision state S_{n-1}, W_n,i(x) = S_{n-1},i(x - c_i) (WPULL = true),
// so that a recomputed segment needs one fused pass per state.
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

static dim3 adj_block(int nx) {
    int bx = nx >= 256 ? 256 : (nx >= 128 ? 128 : 64);
    return dim3(bx, 256 / bx, 1);
}

int adjoint_blocks(int nx, int ny, int nz) {
    dim3 blk = adj_block(nx);
    return ((nx + blk.x - 1) / blk.x) * ((ny + blk.y - 1) / blk.y) * nz;
}

template <int Q, int MODE, int FIELD>
static hipError_t adj_f(bool wpull, const void* Wn, const void* l1, void* l0, const KParams& p, double* partials,
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
                        bool accumulate, hipStream_t s) {
    if (p.field_mode == kFieldUniform) return adj_f<Q, MODE, kFieldUniform>(wpull, Wn, l1, l0, p, partials, accumulate, s);
    if (p.field_mode == kFieldMap) return adj_f<Q, MODE, kFieldMap>(wpull, Wn, l1, l0, p, partials, accumulate, s);
    return adj_f<Q, MODE, kFieldNone>(wpull, Wn, l1, l0, p, partials, accumulate, s);
}

hipError_t launch_adjoint(int Q, int mode, bool wpull, const void* Wn, const void* lam_next, void* lam_n,
                          const KParams& p, double* partials, bool accumulate, hipStream_t s) {
    if (Q == 9) return mode == kF64 ? adj_q<9, kF64>(wpull, Wn, lam_next, lam_n, p, partials, accumulate, s)
                                    : adj_q<9, kF32>(wpull, Wn, lam_next, lam_n, p, partials, accumulate, s);
    return mode == kF64 ? adj_q<19, kF64>(wpull, Wn, lam_next, lam_n, p, partials, accumulate, s)
                        : adj_q<19, kF32>(wpull, Wn, lam_next, lam_n, p, partials, accumulate, s);
}

}  // namespace mlbm
