// Fused pull-stream + BGK collision of the matrix-valued quantum lattice
// Boltzmann method (Sec. 3.3), and its collide-only / stream-only parts.
//
// Organisation (one workgroup = BX consecutive x-cells of one row, 4 waves
// per 64 cells): wave group k owns Pauli channel k of those cells.  Every
// wave gathers the values S_ik(x - c_i) of its channel written by the
// previous pass (Eq. TransportStep read backwards).  The trace wave (k = 0)
// also computes the moments of the gathered pre-collision populations
// (Eq. DiscrAvr) and the factor q_i = omega w_i P_i of Eq. WeqAlgo, and hands
// q_i to the other waves through LDS.  After one barrier each wave applies the
// collision of Eq. CollisionStep to its own channel,
//     S_ik = (1 - omega) a_ik + q_i rho_k,   rho_k = sum_i a_ik,
// which is exact because P_i is a scalar multiplying all four Pauli
// components of rho and u, eps depend on traces only.
//
// Memory: every stored value is read once and written once per pass
// (2 * 4 * Q * sizeof(T) bytes per cell).  Each wave streams only the Q
// segments of its channel; the row index and the channel are uniform across
// a wave, so per-lane addresses are a scalar base plus x.  Stores are
// non-temporal (the field is not re-read within the pass) unless a field is
// small enough for the next pass to find it in the last-level cache (NTS).
// The plain kernels run with a capped number of resident workgroups per CU
// (see step_launch and lds_for_cap).
//
// Template options of k_step: FIELD adds the exact magnetic precession of
// the Bloch channels after the collision (Sec. 5); VAR selects the isothermal
// equilibrium (Sec. 3.1) and/or the positivity-limited rate (Sec. 3.3).  Both
// exchange more data between the waves through LDS and add barriers.  PUSH
// (fused pass only) writes each collided value to x + c_i, where the next
// streaming would take it, so that the last pass of a run of steps leaves the
// pre-collision state without a separate stream-only pass.
#include <map>
#include <mutex>
#include <utility>

#include "block_order.hpp"
#include "common.hpp"
#include "fermi_device.hpp"
#include "internal.hpp"

namespace mlbm {

// FP32 storage: the float constants (omega w_i, 1 - omega, the Appendix
// coefficients) carry fixed rounding errors, so an uncorrected float
// collision gains or loses a fixed ~1e-8 of the conserved moments every step
// and the global averages drift.  (With FP16 storage the half-precision
// rounding of the stored deviations dominates instead: a cell near a steady
// state rounds the same way step after step, and folding each cell's rounding
// defect into its rest and axis populations, measured, cut the drift by 1.3x
// only while slowing the pass by 40%, so the correction is not applied there.)
// The defect of the float outputs is summed in double and folded back exactly
// (fold_defect):
//   every channel k: mass sum_i (S_ik - a_ik) is removed from the rest population;
//   trace channel: momentum component d is removed through the axis pair
//   (+d, -d) (opposite halves: mass and energy unchanged), and energy through
//   the rest and the 2D axis populations (+dE on the rest, -dE/(2D) on each
//   axis population: mass and momentum unchanged).
// Afterwards the conserved moments of S equal those of a up to one final float
// rounding per value, which has no preferred sign.  ENERGY = false (isothermal
// model, where the collision changes the energy on purpose) corrects mass and
// momentum only.
template <int Q, typename C>
__device__ __forceinline__ void fold_defect(C (&S)[Q], int k, double dm, const double (&dj)[3], double dE) {
    constexpr int D = Lat<Q>::D;
    if (k != 0) {
        S[0] = static_cast<C>(static_cast<double>(S[0]) - dm);
        return;
    }
    S[0] = static_cast<C>(static_cast<double>(S[0]) - dm + dE);
    const double de_axis = dE / (2 * D);
#pragma unroll
    for (int i = 1; i <= 2 * D; ++i) {
        // axis velocities 1..2D come in pairs (+d, -d); i odd is +d
        const int dim = (i - 1) / 2;
        const double sgn = (i & 1) ? -0.5 : 0.5;
        S[i] = static_cast<C>(static_cast<double>(S[i]) - de_axis + sgn * dj[dim]);
    }
}

template <int Q, typename C, bool ENERGY = true>
__device__ __forceinline__ void conserve(C (&S)[Q], const C (&a)[Q], int k) {
    double dm = 0.0, dj[3] = {0.0, 0.0, 0.0}, dE = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double dd = static_cast<double>(S[i]) - static_cast<double>(a[i]);
        dm += dd;
#pragma unroll
        for (int c = 0; c < 3; ++c) dj[c] += Lat<Q>::c(i, c) * dd;
        if constexpr (ENERGY) dE += csq<Q>(i) * dd;
    }
    fold_defect<Q, C>(S, k, dm, dj, dE);
}

// Positivity-limited relaxation (Sec. 3.3, paragraph after the algorithm):
// the largest w in [0, om] for which the collided population
// (1 - w) a + w e keeps its smaller eigenvalue at or above min(0, that of a),
// in Pauli coefficients (eigenvalues (x0 +- |x|)/2).  With
// g(w) = a0 + w d0 - |a + w d|, d = e - a, and m = min(0, g(0)), g is concave,
// so {w >= 0 : g(w) >= m} is an interval [0, w*].  If g(om) >= m the bound is
// om; otherwise w* is where h(w) = (a0 - m + w d0)^2 - |a + w d|^2 first
// crosses zero downward (h has the sign of g - m on [0, w*]): the smallest
// root r in [0, om] of the quadratic with h'(r) < 0.  No such root (only
// possible through rounding) gives the safe bound 0.
template <typename C>
__device__ __forceinline__ C psd_bound(C a0, C a1, C a2, C a3, C e0, C e1, C e2, C e3, C om) {
    const C na = sqrt(a1 * a1 + a2 * a2 + a3 * a3);
    const C m = fmin(C(0), a0 - na);
    const C d0 = e0 - a0, d1 = e1 - a1, d2 = e2 - a2, d3 = e3 - a3;
    const C f0 = a0 + om * d0, f1 = a1 + om * d1, f2 = a2 + om * d2, f3 = a3 + om * d3;
    if (f0 - sqrt(f1 * f1 + f2 * f2 + f3 * f3) >= m) return om;
    const C b0 = a0 - m;
    const C A = d0 * d0 - (d1 * d1 + d2 * d2 + d3 * d3);
    const C B = b0 * d0 - (a1 * d1 + a2 * d2 + a3 * d3);
    const C Cc = fmax(C(0), b0 * b0 - na * na);
    const C disc = B * B - A * Cc;
    if (!(disc >= C(0))) return C(0);
    const C q = -(B + copysign(sqrt(disc), B));
    const C r1 = (A != C(0)) ? q / A : C(-1);
    const C r2 = (q != C(0)) ? Cc / q : C(-1);
    C best = C(-1);
    if (r1 >= C(0) && r1 <= om && A * r1 + B < C(0)) best = r1;
    if (r2 >= C(0) && r2 <= om && A * r2 + B < C(0)) best = (best < C(0)) ? r2 : fmin(best, r2);
    return best < C(0) ? C(0) : best;
}

// Field element x of a row segment.  F64 and F32 keep the segment start in
// scalar registers (load_row / store_row); the FP16-deviation pass indexes per
// lane, since its decode constants already fill the scalar registers (measured
// on MI355X at D3Q19 128^3: 146 against 139 us per pass with scalar starts,
// while F64 gains 1% and F32 3%).  Loads are never streaming here: a
// streaming load of the source slowed the FP64 pass by 4%.
template <int MODE, typename T>
__device__ __forceinline__ T load_field(const T* row, int x) {
    if constexpr (MODE == kF16Dev) return row[x];
    else return load_row<false>(row, x);
}

template <int MODE, bool NT, typename T>
__device__ __forceinline__ void store_field(T v, T* row, int x) {
    if constexpr (MODE == kF16Dev) {
        if constexpr (NT) __builtin_nontemporal_store(v, row + x);
        else row[x] = v;
    } else {
        store_row<NT>(v, row, x);
    }
}

// Field pointers of k_step.  Every pass that streams reads and writes distinct
// fields, so its pointers are restrict-qualified; the collide-only pass may run
// in place (src == dst: mlbm_step with an even step count, mlbm_collide), so
// its pointers are plain.  In place, every element is read and then written by
// the same thread.
template <bool DISTINCT, typename T> struct FieldPtr {
    using in = const T*;
    using out = T*;
};
template <typename T> struct FieldPtr<true, T> {
    using in = const T* __restrict__;
    using out = T* __restrict__;
};

template <int Q, int MODE, bool PULL, bool COLL, int BX, int FIELD, int VAR, bool NTS = true, bool PUSH = false>
__global__ void __launch_bounds__(BX * 4)
k_step(typename FieldPtr<PULL, typename Store<MODE>::T>::in src,
       typename FieldPtr<PULL, typename Store<MODE>::T>::out dst, const KParams p, const int order,
       const FdParams fp) {
    using T = typename Store<MODE>::T;
    using C = typename Store<MODE>::C;
    constexpr int D = Lat<Q>::D;
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

    // source coordinate of a pull along each axis, indexed by c + 1: (x - c) mod n
    const int xs[3] = {xx + 1 == nx ? 0 : xx + 1, xx, xx == 0 ? nx - 1 : xx - 1};
    const int ys[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    int zs[3] = {z, z, z};
    if constexpr (D == 3) {
        zs[0] = z + 1 == nz ? 0 : z + 1;
        zs[2] = z == 0 ? nz - 1 : z - 1;
    }

    T raw[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        size_t srow = row;
        int sx = xx;
        if constexpr (PULL) {
            srow = static_cast<size_t>(zs[Lat<Q>::c(i, 2) + 1]) * ny + ys[Lat<Q>::c(i, 1) + 1];
            sx = xs[Lat<Q>::c(i, 0) + 1];
        }
        raw[i] = load_field<MODE>(src + fidx(Q, nx, srow, k, i, 0), sx);
    }

    if constexpr (!COLL) {
        // Streaming alone: a permutation of the stored values, bit exact.
        if (active) {
#pragma unroll
            for (int i = 0; i < Q; ++i) store_field<MODE, NTS>(raw[i], dst + fidx(Q, nx, row, k, i, 0), x);
        }
        return;
    } else {
        // q_i of the trace wave; with a field the same LDS is reused for the
        // exchange of the three Bloch channels (3 Q BX values).  The
        // positivity variant shares all four channels and w_i P_i, and every
        // wave bounds the rate for a quarter of the velocities.
        constexpr bool kIso = (VAR & kVarIso) != 0, kPos = (VAR & kVarPos) != 0;
        static_assert(VAR == 0 || FIELD == kFieldNone, "variants and the field are exclusive");
        // plain and field kernels: q_i of the trace wave (Q BX values), with a field
        // reused for the exchange of the three Bloch channels (3 Q BX values);
        // positivity: the other three channels of every population for the wave
        // that bounds it (3 Q BX values)
        __shared__ C lds[(FIELD != kFieldNone || kPos ? 3 : 1) * Q * BX];
        __shared__ double rsh[VAR != 0 ? 4 : 1][BX];      // rho_k of the Bloch waves; tr rho
        __shared__ double jsh[VAR != 0 ? 4 : 1][BX];      // the trace wave's j (3 components) and K
        __shared__ double esh[kIso ? 2 : 1][BX];          // isothermal: F_{d/2}(nu) per eigen-channel
        __shared__ C pmin[kPos ? 4 : 1][BX];              // positivity: each wave's bound on the rate
        C (*qs)[BX] = reinterpret_cast<C (*)[BX]>(lds);
        C a[Q];
        double rk = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            a[i] = decode<MODE>(raw[i], k, i, p);
            rk += static_cast<double>(a[i]);
        }
        // moments (Eq. DiscrAvr) in double; sums over c_i in {0, +-1}
        auto trace_moments = [&](double& J0, double& J1, double& J2, double& K) {
            J0 = J1 = J2 = K = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double v = static_cast<double>(a[i]);
                if (Lat<Q>::c(i, 0) == 1) J0 += v; else if (Lat<Q>::c(i, 0) == -1) J0 -= v;
                if (Lat<Q>::c(i, 1) == 1) J1 += v; else if (Lat<Q>::c(i, 1) == -1) J1 -= v;
                if (Lat<Q>::c(i, 2) == 1) J2 += v; else if (Lat<Q>::c(i, 2) == -1) J2 -= v;
                if (csq<Q>(i) == 1) K += v; else if (csq<Q>(i) == 2) K += 2.0 * v;
            }
        };
        // polynomial factor (Eq. WeqAlgo, Appendix), with v = beta0 xi u so that
        // beta0 e_i.u = c_i.v:
        //   P_i = alpha1 + alpha5 beta0 |u|^2/2 + alpha2 beta0 xi^2 |c_i|^2 / 2
        //         + (c_i.v)(alpha3 + alpha4 c_i.v)
        struct PCoef { C A, B, v0, v1, v2; };
        auto p_coef = [&](double T, double J0, double J1, double J2, double K, double eps_iso) {
            const double invT = 1.0 / T;
            const double u0 = p.xi * J0 * invT, u1 = p.xi * J1 * invT, u2 = (D == 3) ? p.xi * J2 * invT : 0.0;
            const double uu = u0 * u0 + u1 * u1 + u2 * u2;
            const double eps = kIso ? eps_iso : p.half_xi2 * K * invT - 0.5 * uu;
            const double b = p.beta0 * eps;
            return PCoef{static_cast<C>(p.a1_0 + p.a1_b * b + p.a5 * p.beta0 * 0.5 * uu),
                         static_cast<C>((p.a2_0 + p.a2_b * b) * p.beta0 * p.half_xi2),
                         static_cast<C>(p.beta0 * p.xi * u0), static_cast<C>(p.beta0 * p.xi * u1),
                         static_cast<C>(p.beta0 * p.xi * u2)};
        };
        auto p_of = [&](const PCoef& q, int i) {
            const C a3 = cst<C>(p.a3, p.a3f), a4 = cst<C>(p.a4, p.a4f);
            C cv = C(0);
            if (Lat<Q>::c(i, 0) == 1) cv += q.v0; else if (Lat<Q>::c(i, 0) == -1) cv -= q.v0;
            if (Lat<Q>::c(i, 1) == 1) cv += q.v1; else if (Lat<Q>::c(i, 1) == -1) cv -= q.v1;
            if (Lat<Q>::c(i, 2) == 1) cv += q.v2; else if (Lat<Q>::c(i, 2) == -1) cv -= q.v2;
            C P = q.A + cv * (a3 + a4 * cv);
            if (csq<Q>(i) == 1) P += q.B; else if (csq<Q>(i) == 2) P += C(2) * q.B;
            return P;
        };
        const C r = static_cast<C>(rk);
        C S[Q];
        if constexpr (VAR == 0) {
            // the trace wave builds q_i = omega w_i P_i for all four channels
            if (k == 0) {
                double J0, J1, J2, K;
                trace_moments(J0, J1, J2, K);
                const PCoef q = p_coef(rk, J0, J1, J2, K, 0.0);
#pragma unroll
                for (int i = 0; i < Q; ++i) qs[i][lx] = omw_of<C>(p, i) * p_of(q, i);
            }
            __syncthreads();
            // collision (Eq. CollisionStep) of this wave's channel
            const C omm = cst<C>(p.one_m_om, p.one_m_omf);
#pragma unroll
            for (int i = 0; i < Q; ++i) S[i] = omm * a[i] + qs[i][lx] * r;
        } else {
            // Variants: every wave forms the cell's coefficients of P_i itself from the
            // trace moments and rho_k shared through LDS, so the only barriers are the
            // exchange itself, the isothermal inversion and the positivity bound.
            if (k > 0) rsh[k - 1][lx] = rk;
            else rsh[3][lx] = rk;
            if (k == 0) {
                double J0, J1, J2, K;
                trace_moments(J0, J1, J2, K);
                jsh[0][lx] = J0;
                jsh[1][lx] = J1;
                jsh[2][lx] = J2;
                jsh[3][lx] = K;
            }
            // positivity: wave i mod 4 bounds population i; it holds channel i mod 4 of
            // it and reads the other three from slot 3 i + (rank of the channel among them)
            C (*ab)[BX] = reinterpret_cast<C (*)[BX]>(lds);
            auto slot = [](int i, int kk) { const int b = i & 3; return 3 * i + (kk < b ? kk : kk - 1); };
            if constexpr (kPos) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if ((i & 3) != k) ab[slot(i, k)][lx] = a[i];
                }
            }
            __syncthreads();
            const double T = rsh[3][lx];
            double eps_iso = 0.0;
            if constexpr (kIso) {
                // isothermal model: the Fermi-Dirac state at beta = beta0 with the
                // cell's density matrix; its eigen-channels (tr rho +- |rho|)/2 are
                // inverted by waves 1 (up) and 2 (down) side by side
                const double rv = sqrt(rsh[0][lx] * rsh[0][lx] + rsh[1][lx] * rsh[1][lx] + rsh[2][lx] * rsh[2][lx]);
                if (k == 1 || k == 2) {
                    const double n = 0.5 * (T + (k == 1 ? rv : -rv));
                    esh[k - 1][lx] = fd::iso_channel<D>(p.beta0, n, fp);
                }
                __syncthreads();
                eps_iso = fd::iso_energy<D>(p.beta0, 0.5 * (T + rv), 0.5 * (T - rv), esh[0][lx], esh[1][lx]);
            }
            const PCoef q = p_coef(T, jsh[0][lx], jsh[1][lx], jsh[2][lx], jsh[3][lx], eps_iso);
            C omm, omc = C(0);
            if constexpr (kPos) {
                // the largest rate in [0, omega] keeping every population's smaller
                // eigenvalue at or above min(0, its value): wave k bounds velocities
                // i = k mod 4, and the cell's rate is the minimum of the four bounds;
                // the equilibrium of population i is w_i P_i rho (Eq. WeqAlgo)
                const C r0 = static_cast<C>(rsh[3][lx]), r1 = static_cast<C>(rsh[0][lx]),
                        r2 = static_cast<C>(rsh[1][lx]), r3 = static_cast<C>(rsh[2][lx]);
                const C om = static_cast<C>(p.om);
                C m = om;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if ((i & 3) == k) {
                        C ai[4];
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) ai[kk] = (kk == k) ? a[i] : ab[slot(i, kk)][lx];
                        const C wPi = static_cast<C>(p.w[i]) * p_of(q, i);
                        m = fmin(m, psd_bound<C>(ai[0], ai[1], ai[2], ai[3], wPi * r0, wPi * r1, wPi * r2, wPi * r3, om));
                    }
                }
                pmin[k][lx] = m;
                __syncthreads();
                omc = fmin(fmin(pmin[0][lx], pmin[1][lx]), fmin(pmin[2][lx], pmin[3][lx]));
                omm = C(1) - omc;
            } else {
                omm = cst<C>(p.one_m_om, p.one_m_omf);
            }
            // collision (Eq. CollisionStep) of this wave's channel
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if constexpr (kPos) S[i] = omm * a[i] + (omc * (static_cast<C>(p.w[i]) * p_of(q, i))) * r;
                else S[i] = omm * a[i] + (omw_of<C>(p, i) * p_of(q, i)) * r;
            }
        }
        if constexpr (MODE == kF32) conserve<Q, C, !kIso>(S, a, k);
        if constexpr (FIELD != kFieldNone) {
            // magnetic precession of the Bloch components; it commutes with the
            // BGK collision cell by cell, so applying it afterwards is exact
            C (*sb)[Q][BX] = reinterpret_cast<C (*)[Q][BX]>(lds);
            __syncthreads();          // every wave has read qs
            if (k > 0) {
#pragma unroll
                for (int i = 0; i < Q; ++i) sb[k - 1][i][lx] = S[i];
            }
            __syncthreads();
            if (k > 0) {
                double rr[3];
                if constexpr (FIELD == kFieldUniform) {
#pragma unroll
                    for (int l = 0; l < 3; ++l) rr[l] = p.rot[(k - 1) * 3 + l];
                } else {
                    const size_t cell = row * nx + xx;
                    const size_t N = static_cast<size_t>(p.ncell);
                    const double b[3] = {p.bmap[cell], p.bmap[N + cell], p.bmap[2 * N + cell]};
                    rotation_row(b, k - 1, rr);
                }
                const C r0 = static_cast<C>(rr[0]), r1 = static_cast<C>(rr[1]), r2 = static_cast<C>(rr[2]);
#pragma unroll
                for (int i = 0; i < Q; ++i) S[i] = r0 * sb[0][i][lx] + r1 * sb[1][i][lx] + r2 * sb[2][i][lx];
            }
        }
        if (active) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                size_t drow = row;
                int dx = x;
                if constexpr (PUSH) {
                    // the streaming of the step as well (Eq. TransportStep): the value leaves for x + c_i
                    drow = static_cast<size_t>(zs[1 - Lat<Q>::c(i, 2)]) * ny + ys[1 - Lat<Q>::c(i, 1)];
                    dx = xs[1 - Lat<Q>::c(i, 0)];
                }
                store_field<MODE, NTS>(encode<MODE>(S[i], k, i, p), dst + fidx(Q, nx, drow, k, i, 0), dx);
            }
        }
    }
}

// Launch shape (cells per workgroup along x, block order, resident
// workgroups per CU) when the handle does not fix one, from sweeps on MI355X
// (fused-pass bandwidth measured through mlbm_step).  D2Q9 grids below 2^20
// cells, whose fields stay in the caches: 64-cell blocks, one row range per
// XCD, no cap.  Otherwise:
//   FP64: 64-cell blocks with at most 2 workgroups per CU for D3Q19 above 64^3
//     (128^3: 6.00 TB/s against 5.65 uncapped; 384^3 with one row range per
//     XCD: 5.73 against 5.54 for the best uncapped shape), 3 per CU for
//     smaller D3Q19 grids and for D2Q9 (1024^2, 8-row interleave: 6.10 TB/s
//     against 5.95); natural order below 2^24 cells, per-XCD ranges above;
//   FP32: D3Q19 up to 2^24 cells 64-cell blocks, 8-row interleave, 3 per CU
//     from 128^3 on (6.03 against 5.93 TB/s); larger D3Q19 grids 128-cell
//     blocks, per-XCD ranges; D2Q9 128-cell blocks, 8-row interleave;
//   FP16: as FP32 without a cap (it gains nothing there).
// Field writes are temporal when one field holds at most 192 MiB and
// streaming above.  The threshold is an empirical cut-off between measured
// per-pass times, not a capacity bound: the two fields of a pass can together
// exceed the 256 MB last-level cache below it (D2Q9 1024^2 FP32: 151 MB per
// field), and part of what the next pass reads is still found there.
// Temporal: D2Q9 512^2 FP32 13.7 against 15.8 us per pass, D3Q19 64^3 FP32
// 26.0 against 29.9 us, D2Q9 1024^2 FP32 48.7 against 50.6 us.  Streaming:
// D3Q19 128^3 FP64 (1.27 GB per field) 424 against 445 us, D2Q9 1024^2 FP64
// (302 MB) 98 against 102 us.
// The magnetic-field kernels (more LDS) and the isothermal and positivity
// kernels (more arithmetic per cell) always stream their stores, the variants
// run in 64-cell blocks, and they take their own order and cap: measured per
// kind at D3Q19 128^3 FP64 (fused-pass medians of five runs, against the
// uncapped natural order): isothermal 8-row interleave with 3 workgroups per
// CU (426 against 451 us), positivity natural order with 3 (429 against
// 441), both together uncapped (443), uniform field 8-row interleave with 2
// (426 against 433), per-cell field map 8-row interleave with 3 (437 against
// 471).  Elsewhere they run uncapped in the plain kernels' order.
LaunchCfg step_launch(int nx, int ny, int nz, int Q, int mode, int variant, int field_mode, LaunchCfg want) {
    LaunchCfg c = want;
    const double cells = static_cast<double>(nx) * ny * nz;
    if (c.stores < 0) {
        const double field_bytes = 4.0 * Q * cells * (mode == kF64 ? 8 : (mode == kF32 ? 4 : 2));
        c.stores = field_bytes <= 192.0 * 1048576.0 ? 1 : 0;
    }
    const bool big3d = Q == 19 && cells >= 16777216.0 && nx > 64;
    if (variant != 0 || field_mode != kFieldNone) {
        LaunchCfg plain = want;
        plain.order = -1;
        plain = step_launch(nx, ny, nz, Q, mode, 0, kFieldNone, plain);
        if (variant != 0) c.bx = 64;                    // the variant kernels exist for 64-cell blocks only
        else if (c.bx == 0) c.bx = plain.bx;
        c.stores = 0;
        const bool measured = Q == 19 && mode == kF64 && cells > 262144.0 && !big3d;
        int order = plain.order, cap = 0;
        if (measured) {
            if (variant == kVarIso) { order = kOrderInterleave8; cap = 3; }
            else if (variant == kVarPos) { order = kOrderNatural; cap = 3; }
            else if (variant == (kVarIso | kVarPos)) { order = kOrderNatural; cap = 0; }
            else if (field_mode == kFieldUniform) { order = kOrderInterleave8; cap = 2; }
            else if (field_mode == kFieldMap) { order = kOrderInterleave8; cap = 3; }
        }
        if (c.order < 0) c.order = order;
        if (c.cap < 0) c.cap = cap;
        return c;
    }
    if (Q == 9 && cells < 1048576.0) {
        // D2Q9 below 2^20 cells: one contiguous row range per XCD, no cap (512^2: FP64 23.0 against
        // 24.6 us per pass, FP32 13.1 against 13.7; 64^2 FP64 3.3 against 3.7)
        if (c.bx == 0) c.bx = 64;
        if (c.order < 0) c.order = kOrderXcdRange;
        if (c.cap < 0) c.cap = 0;
        return c;
    }
    if (mode == kF64) {
        if (c.bx == 0) c.bx = 64;
        if (c.order < 0) c.order = (Q == 9) ? kOrderInterleave8 : (big3d ? kOrderXcdRange : kOrderNatural);
        if (c.cap < 0) c.cap = (Q == 19 && cells > 262144.0) ? 2 : 3;
    } else {
        if (c.bx == 0) c.bx = ((Q == 9 && nx >= 128) || big3d) ? 128 : 64;
        if (c.order < 0) c.order = big3d ? kOrderXcdRange : kOrderInterleave8;
        if (c.cap < 0) c.cap = (mode == kF32 && Q == 19 && !big3d && cells >= 2097152.0) ? 3 : 0;
    }
    return c;
}

// Dynamic LDS that limits a kernel to `cap` resident workgroups per CU.
// Fewer waves in flight means fewer concurrent DRAM streams (every wave
// gathers Q segments and writes Q segments), which on MI355X raises the
// bandwidth the pass reaches; the LDS is reserved, never touched.  The size is
// the smallest one at which the runtime's occupancy calculator reports at
// most `cap` workgroups, found once per kernel and cap and cached.
size_t lds_for_cap(const void* fn, int threads, int cap) {
    if (cap <= 0) return 0;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(fn, cap);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    auto occupancy = [&](size_t dyn) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, dyn) != hipSuccess) return -1;
        return n;
    };
    hipFuncAttributes attr{};
    size_t hi = 0;
    if (hipFuncGetAttributes(&attr, fn) == hipSuccess)
        hi = attr.maxDynamicSharedSizeBytes > 0 ? static_cast<size_t>(attr.maxDynamicSharedSizeBytes)
                                                : 65536 - attr.sharedSizeBytes;
    size_t dyn = 0;
    const int n0 = occupancy(0);
    if (n0 > cap && hi > 0 && occupancy(hi) >= 0) {
        size_t lo = 0;
        while (lo < hi) {          // smallest dyn with occupancy <= cap (occupancy falls as dyn grows)
            const size_t mid = lo + (hi - lo) / 2;
            const int n = occupancy(mid);
            if (n >= 0 && n <= cap) hi = mid;
            else lo = mid + 1;
        }
        dyn = lo;
    }
    (void)hipGetLastError();      // the queries leave no error behind
    cache.emplace(key, dyn);
    return dyn;
}

template <int Q, int MODE, bool PULL, bool COLL, int FIELD, int VAR = 0, bool PUSH = false>
static hipError_t launch(const void* src, void* dst, const KParams& p, const FdParams& fp, LaunchCfg c,
                         hipStream_t s) {
    using T = typename Store<MODE>::T;
    if constexpr (VAR != 0) c.bx = 64;        // the variants are built for 64-cell blocks only
    // only the plain kernels write temporally (step_launch streams the others)
    constexpr bool kPlain = VAR == 0 && FIELD == kFieldNone;
    const bool temporal = kPlain && c.stores == 1;
    const dim3 grd(static_cast<unsigned>((p.nx + c.bx - 1) / c.bx) * p.ny * p.nz);
    if (c.bx == 64) {
        const auto fn = temporal ? k_step<Q, MODE, PULL, COLL, 64, FIELD, VAR, !kPlain, PUSH>
                                 : k_step<Q, MODE, PULL, COLL, 64, FIELD, VAR, true, PUSH>;
        const size_t dyn = lds_for_cap(reinterpret_cast<const void*>(fn), 256, c.cap);
        hipLaunchKernelGGL(fn, grd, dim3(64, 4), dyn, s, static_cast<const T*>(src), static_cast<T*>(dst), p,
                           c.order, fp);
    } else if constexpr (VAR == 0) {
        const auto fn = temporal ? k_step<Q, MODE, PULL, COLL, 128, FIELD, 0, !kPlain, PUSH>
                                 : k_step<Q, MODE, PULL, COLL, 128, FIELD, 0, true, PUSH>;
        const size_t dyn = lds_for_cap(reinterpret_cast<const void*>(fn), 512, c.cap);
        hipLaunchKernelGGL(fn, grd, dim3(128, 4), dyn, s, static_cast<const T*>(src), static_cast<T*>(dst), p,
                           c.order, fp);
    }
    return hipGetLastError();
}

template <int Q, int MODE, bool PULL, bool PUSH = false>
static hipError_t launch_coll(const void* src, void* dst, const KParams& p, const FdParams& fp, LaunchCfg c,
                              hipStream_t s) {
    if (p.variant == kVarIso) return launch<Q, MODE, PULL, true, kFieldNone, kVarIso, PUSH>(src, dst, p, fp, c, s);
    if (p.variant == kVarPos) return launch<Q, MODE, PULL, true, kFieldNone, kVarPos, PUSH>(src, dst, p, fp, c, s);
    if (p.variant == (kVarIso | kVarPos))
        return launch<Q, MODE, PULL, true, kFieldNone, kVarIso | kVarPos, PUSH>(src, dst, p, fp, c, s);
    if (p.field_mode == kFieldUniform)
        return launch<Q, MODE, PULL, true, kFieldUniform, 0, PUSH>(src, dst, p, fp, c, s);
    if (p.field_mode == kFieldMap) return launch<Q, MODE, PULL, true, kFieldMap, 0, PUSH>(src, dst, p, fp, c, s);
    return launch<Q, MODE, PULL, true, kFieldNone, 0, PUSH>(src, dst, p, fp, c, s);
}

template <int Q, int MODE>
static hipError_t dispatch_kind(StepKind kind, const void* src, void* dst, const KParams& p, const FdParams& fp,
                                LaunchCfg c, hipStream_t s) {
    switch (kind) {
        case StepKind::Fused: return launch_coll<Q, MODE, true>(src, dst, p, fp, c, s);
        case StepKind::FusedPush: return launch_coll<Q, MODE, true, true>(src, dst, p, fp, c, s);
        case StepKind::CollideOnly: return launch_coll<Q, MODE, false>(src, dst, p, fp, c, s);
        case StepKind::StreamOnly: return launch<Q, MODE, true, false, kFieldNone>(src, dst, p, fp, c, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(StepKind kind, int Q, int mode, const void* src, void* dst, const KParams& p,
                       const FdParams& fp, LaunchCfg want, hipStream_t s) {
    // the stream-only pass runs the plain kernel whatever the collision
    const bool stream_only = kind == StepKind::StreamOnly;
    LaunchCfg c = step_launch(p.nx, p.ny, p.nz, Q, mode, stream_only ? 0 : p.variant,
                              stream_only ? static_cast<int>(kFieldNone) : p.field_mode, want);
    // The pushing pass writes every value one cell on in x, so a 64-cell chunk fills the cache
    // lines at its two ends only partly and the neighbouring chunk fills the rest.  When a row
    // has at most 128 cells one 128-cell chunk covers it and writes every line of its destination
    // rows whole.  Measured at D3Q19 128^3: the pushing pass FP64 463 against 543-564 us with 1
    // workgroup per CU, FP16 116 against 137-140 us uncapped, FP32 244-247 against 250 us
    // (mlbm_step(20): FP64 421-423 against 427 us per step).  Longer rows keep the step's shape:
    // there the 128-cell chunks still split lines and measured slower (D3Q19 384^3 FP16
    // mlbm_step(20) 3 074 against 3 011 us per step, D2Q9 1024^2 FP32 49.3 against 47.9 us).
    if (kind == StepKind::FusedPush && p.variant == 0 && p.field_mode == kFieldNone && p.nx > 64 && p.nx <= 128) {
        if (want.bx == 0) c.bx = 128;
        if (want.order < 0) c.order = kOrderNatural;
        if (want.cap < 0) c.cap = (mode == kF64 && Q == 19) ? 1 : 0;
    }
    if (Q == 9) {
        if (mode == kF64) return dispatch_kind<9, kF64>(kind, src, dst, p, fp, c, s);
        if (mode == kF32) return dispatch_kind<9, kF32>(kind, src, dst, p, fp, c, s);
        return dispatch_kind<9, kF16Dev>(kind, src, dst, p, fp, c, s);
    }
    if (mode == kF64) return dispatch_kind<19, kF64>(kind, src, dst, p, fp, c, s);
    if (mode == kF32) return dispatch_kind<19, kF32>(kind, src, dst, p, fp, c, s);
    return dispatch_kind<19, kF16Dev>(kind, src, dst, p, fp, c, s);
}

}  // namespace mlbm
