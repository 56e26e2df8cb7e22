// Fused pull-stream + BGK collision of the matrix-valued quantum lattice
// Boltzmann method (Sec. 3.3), and its collide-only / stream-only parts.
//
// One thread owns one cell x.  In the fused pass it gathers the
// post-collision values S_i(x - c_i) written by the previous pass
// (Eq. TransportStep read backwards), computes the moments of the gathered
// pre-collision populations (Eq. DiscrAvr), the polynomial factor P_i of
// Eq. WeqAlgo and the collision of Eq. CollisionStep, and writes S_i(x).
//
// Structure used to keep registers low: P_i multiplies all four Pauli
// components of rho, and u, eps depend on traces only, so the trace channel
// (k = 0) is processed first; it yields q_i = omega w_i P_i.  Each Bloch
// channel k = 1..3 is then independent and linear:
//     S_ik = (1 - omega) a_ik + q_i rho_k,   rho_k = sum_i a_ik.
//
// Memory: every stored value is read once and written once per pass
// (2 * 4 * Q * sizeof(T) bytes per cell); neighbouring lanes read
// neighbouring addresses of the same plane, shifted by at most one element.
#include "common.hpp"
#include "internal.hpp"

namespace mlbm {

template <int Q, int MODE, bool PULL, bool COLL>
__global__ void __launch_bounds__(256)
k_step(const typename Store<MODE>::T* __restrict__ src, typename Store<MODE>::T* __restrict__ dst,
       const KParams p) {
    using T = typename Store<MODE>::T;
    using C = typename Store<MODE>::C;
    constexpr int D = Lat<Q>::D;

    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= p.nx || y >= p.ny) return;
    const int nxy = p.nx * p.ny;
    const int node = x + p.nx * y + nxy * z;
    const size_t N = static_cast<size_t>(p.ncell);

    int sn[Q];
    if constexpr (PULL) {
        int xo[3], yo[3], zo[3];
        pull_coords(x, p.nx, 1, xo);
        pull_coords(y, p.ny, p.nx, yo);
        if constexpr (D == 3) {
            pull_coords(z, p.nz, nxy, zo);
        } else {
            zo[0] = zo[1] = zo[2] = 0;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i)
            sn[i] = xo[Lat<Q>::c(i, 0) + 1] + yo[Lat<Q>::c(i, 1) + 1] + zo[Lat<Q>::c(i, 2) + 1];
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) sn[i] = node;
    }

    if constexpr (!COLL) {
        // Streaming alone: a permutation of the stored values, bit exact.
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T v[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = src[(k * Q + i) * N + sn[i]];
#pragma unroll
            for (int i = 0; i < Q; ++i) dst[(k * Q + i) * N + node] = v[i];
        }
        return;
    }

    // ---- trace channel: moments (Eq. DiscrAvr) in double ----------------
    C a[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) a[i] = decode<MODE>(src[i * N + sn[i]], 0, i, p);
    double T0 = 0.0, J0 = 0.0, J1 = 0.0, J2 = 0.0, K = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = static_cast<double>(a[i]);
        T0 += v;
        if (Lat<Q>::c(i, 0) == 1) J0 += v; else if (Lat<Q>::c(i, 0) == -1) J0 -= v;
        if (Lat<Q>::c(i, 1) == 1) J1 += v; else if (Lat<Q>::c(i, 1) == -1) J1 -= v;
        if (Lat<Q>::c(i, 2) == 1) J2 += v; else if (Lat<Q>::c(i, 2) == -1) J2 -= v;
        if (csq<Q>(i) == 1) K += v; else if (csq<Q>(i) == 2) K += 2.0 * v;
    }
    const double invT = 1.0 / T0;
    const double u0 = p.xi * J0 * invT, u1 = p.xi * J1 * invT, u2 = (D == 3) ? p.xi * J2 * invT : 0.0;
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    const double eps = p.half_xi2 * K * invT - 0.5 * uu;

    // ---- polynomial factor P_i (Eq. WeqAlgo, Appendix) ------------------
    //   P_i = alpha1 + alpha2 beta0 |e_i|^2/2 + alpha3 (c_i.v) + alpha4 (c_i.v)^2
    //         + alpha5 beta0 |u|^2/2,   v = beta0 xi u  (so beta0 e_i.u = c_i.v)
    const double b = p.beta0 * eps;
    const C A = static_cast<C>(p.a1_0 + p.a1_b * b + p.a5 * p.beta0 * 0.5 * uu);
    const C B = static_cast<C>((p.a2_0 + p.a2_b * b) * p.beta0 * p.half_xi2);
    const C v0 = static_cast<C>(p.beta0 * p.xi * u0);
    const C v1 = static_cast<C>(p.beta0 * p.xi * u1);
    const C v2 = static_cast<C>(p.beta0 * p.xi * u2);
    const C a3 = cst<C>(p.a3, p.a3f), a4 = cst<C>(p.a4, p.a4f);
    const C omm = cst<C>(p.one_m_om, p.one_m_omf);
    C q[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        C cv = C(0);
        if (Lat<Q>::c(i, 0) == 1) cv += v0; else if (Lat<Q>::c(i, 0) == -1) cv -= v0;
        if (Lat<Q>::c(i, 1) == 1) cv += v1; else if (Lat<Q>::c(i, 1) == -1) cv -= v1;
        if (Lat<Q>::c(i, 2) == 1) cv += v2; else if (Lat<Q>::c(i, 2) == -1) cv -= v2;
        C P = A + cv * (a3 + a4 * cv);
        if (csq<Q>(i) == 1) P += B; else if (csq<Q>(i) == 2) P += C(2) * B;
        q[i] = omw_of<C>(p, i) * P;
    }

    // ---- collision (Eq. CollisionStep), trace channel --------------------
    {
        const C r0 = static_cast<C>(T0);
#pragma unroll
        for (int i = 0; i < Q; ++i) dst[i * N + node] = encode<MODE>(omm * a[i] + q[i] * r0, 0, i, p);
    }
    // ---- Bloch channels ----------------------------------------------------
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        C b_[Q];
        double rk = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            b_[i] = decode<MODE>(src[(k * Q + i) * N + sn[i]], k, i, p);
            rk += static_cast<double>(b_[i]);
        }
        const C r = static_cast<C>(rk);
#pragma unroll
        for (int i = 0; i < Q; ++i) dst[(k * Q + i) * N + node] = encode<MODE>(omm * b_[i] + q[i] * r, k, i, p);
    }
}

// Block shape: x-extent from {256, 128, 64} with the least idle lanes
// (ties to the wider), y-extent filling 256 threads.
static dim3 step_block(int nx) {
    int best = 256;
    long best_waste = -1;
    for (int bx : {256, 128, 64}) {
        long chunks = (nx + bx - 1) / bx;
        long waste = chunks * bx - nx;
        if (best_waste < 0 || waste < best_waste) { best = bx; best_waste = waste; }
    }
    return dim3(best, 256 / best, 1);
}

template <int Q, int MODE, bool PULL, bool COLL>
static hipError_t launch(const void* src, void* dst, const KParams& p, hipStream_t s) {
    using T = typename Store<MODE>::T;
    dim3 blk = step_block(p.nx);
    dim3 grd((p.nx + blk.x - 1) / blk.x, (p.ny + blk.y - 1) / blk.y, p.nz);
    hipLaunchKernelGGL((k_step<Q, MODE, PULL, COLL>), grd, blk, 0, s, static_cast<const T*>(src),
                       static_cast<T*>(dst), p);
    return hipGetLastError();
}

template <int Q, int MODE>
static hipError_t dispatch_kind(StepKind kind, const void* src, void* dst, const KParams& p, hipStream_t s) {
    switch (kind) {
        case StepKind::Fused: return launch<Q, MODE, true, true>(src, dst, p, s);
        case StepKind::CollideOnly: return launch<Q, MODE, false, true>(src, dst, p, s);
        case StepKind::StreamOnly: return launch<Q, MODE, true, false>(src, dst, p, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(StepKind kind, int Q, int mode, const void* src, void* dst, const KParams& p,
                       hipStream_t s) {
    if (Q == 9) {
        if (mode == kF64) return dispatch_kind<9, kF64>(kind, src, dst, p, s);
        if (mode == kF32) return dispatch_kind<9, kF32>(kind, src, dst, p, s);
        return dispatch_kind<9, kF16Dev>(kind, src, dst, p, s);
    }
    if (mode == kF64) return dispatch_kind<19, kF64>(kind, src, dst, p, s);
    if (mode == kF32) return dispatch_kind<19, kF32>(kind, src, dst, p, s);
    return dispatch_kind<19, kF16Dev>(kind, src, dst, p, s);
}

}  // namespace mlbm
