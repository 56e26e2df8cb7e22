// Host-side declarations shared by the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace mlbm {

// Fused: pull-stream then collide; FusedPush: the same, with every collided value
// written where the next streaming sends it (x + c_i), so that its output is the
// pre-collision state after the following streaming (src and dst distinct).
enum class StepKind { Fused, CollideOnly, StreamOnly, FusedPush };

// Launch shape of the step kernels: cells per workgroup along x (64 or 128;
// 0 = automatic) and block order (-1 = automatic).
enum { kOrderNatural = 0, kOrderXcdRange = 1, kOrderInterleave8 = 2 };
struct LaunchCfg {
    int bx = 0;
    int order = -1;
    int cap = -1;      // workgroups resident per CU: -1 automatic, 0 hardware limit, > 0 at most that many
    int stores = -1;   // field writes: -1 automatic, 0 streaming (non-temporal), 1 temporal
};
LaunchCfg step_launch(int nx, int ny, int nz, int Q, int mode, int variant, int field_mode, LaunchCfg want);

// Dynamic LDS that holds a kernel (launched with `threads` threads per
// workgroup) to at most `cap` resident workgroups per CU; 0 for cap <= 0.
size_t lds_for_cap(const void* fn, int threads, int cap);

// Gauss-Legendre rule on [-1, 1] used by the device Fermi-Dirac integrals.
constexpr int kGL = 20;
struct FdParams {
    double gl_x[kGL];
    double gl_w[kGL];
};

hipError_t launch_step(StepKind kind, int Q, int mode, const void* src, void* dst, const KParams& p,
                       const FdParams& fp, LaunchCfg want, hipStream_t s);

// Eigen-channel variant of the fused / collide-only pass (double storage only).
hipError_t launch_step_eigen(StepKind kind, int Q, const void* src, void* dst, const KParams& p,
                             const FdParams& fp, double* partials, hipStream_t s);

// Per-cell moments and block partial sums.  partials: kRedBlocks x kRedSlots.
//   slots 0..3 sum of rho_k, 4..6 sum of tr(rho) u, 7 sum of total energy,
//   8 number of populations with a negative eigenvalue, 9 number of
//   non-finite values.
hipError_t launch_moments(int Q, int mode, const void* W, double* rho4, double* u, double* eps,
                          const KParams& p, double* partials, hipStream_t s);

// Spin loss: slot 0 partial sum of |r - r_target|^2; optional adjoint seed.
hipError_t launch_relaxation(int Q, int mode, const void* W, const double* g, const KParams& p, double* partials,
                             hipStream_t s);
hipError_t launch_spin_loss(int Q, int mode, const void* W, const double* r_target, void* lam,
                            const KParams& p, double* partials, hipStream_t s);

// Launch shape of the adjoint kernels: the form (kAdjAuto, kAdjChannel: one
// wave per Pauli channel on row-blocked cells like the step passes,
// kAdjCell: one thread per cell with all four channels) and, for the channel
// form, the step kernels' shape parameters (block width, order, cap, stores).
// The magnetic-field adjoint exists in the cell form only.
enum { kAdjAuto = 0, kAdjChannel = 1, kAdjCell = 2 };
struct AdjointCfg {
    int form = kAdjAuto;
    LaunchCfg lc;
};
AdjointCfg adjoint_launch(int nx, int ny, int nz, int Q, int mode, int field_mode, AdjointCfg want);

// Adjoint of one step: one partial of dL/domega per block
// (adjoint_blocks(...) values, stride 1).  With wpull, Wn is the
// previous post-collision state and W_n is gathered from it by a pull.
hipError_t launch_adjoint(int Q, int mode, bool wpull, const void* Wn, const void* lam_next, void* lam_n,
                          const KParams& p, double* partials, bool accumulate, AdjointCfg want, hipStream_t s);

// Initial Fermi-Dirac state.  phase 0: only reduce global sums (slots 0..3
// rho_k, 4..6 tr(rho) u, 7 total energy); phase 1: reduce max |a - R| / w_i
// into slot 0 (max); phase 2: write W.  Slots 8, 9 count domain errors and
// failed inversions in every phase.
// how mlbm_init_* names the per-cell state
enum InitSource { kFromDensity = 0, kFromChemical = 1 };
hipError_t launch_init(int Q, int mode, int phase, int src, void* W, const double* a, const double* axis,
                       const double* u, const double* T, const KParams& p, const FdParams& fp, double* partials,
                       hipStream_t s);

// Reduce nblocks rows of `stride` partials (stride <= kRedSlots) to one
// value per slot in a fixed order.  Bit s of max_mask selects a max instead of
// a sum for slot s.  Slot 0 is multiplied by scale0.  When accumulate_into is
// non-null, only slot 0 is produced and added to *accumulate_into; otherwise
// kRedSlots values go to out (slots >= stride are 0).
hipError_t launch_finalize(const double* partials, int nblocks, int stride, unsigned max_mask, double* out,
                           double* accumulate_into, double scale0, hipStream_t s);

// accumulate_into[0] += scale0 * sum of x[0 .. n), reduced in a fixed order.
// Up to kSumDirect values in one block; longer sums first reduce at most
// kSumChunks consecutive chunks in parallel into tail[0 .. kSumChunks).
constexpr int kSumDirect = 4096;
constexpr int kSumChunks = 1024;
hipError_t launch_sum_into(const double* x, size_t n, double* tail, double* accumulate_into, double scale0,
                           hipStream_t s);

// Number of blocks (= partials) of launch_adjoint for a grid and configuration.
int adjoint_blocks(const KParams& p, int mode, AdjointCfg want);

// Flat copy of n16 16-byte vectors (16-byte aligned, non-overlapping).
hipError_t launch_copy16(const void* src, void* dst, size_t n16, hipStream_t s);

}  // namespace mlbm
