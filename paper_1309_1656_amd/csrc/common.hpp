// Shared device-side definitions: lattice tables, storage codecs, kernel
// parameter block.
//
// Lattices (Sec. 3, Fig. 1; Sec. 3.1): velocities e_i = xi c_i with
// c_i in {-1,0,1}^d, D3Q19 without the eight corners.  The enumeration order
// is the one documented in include/mlbm.h: rest, axis pairs, diagonal pairs,
// each velocity followed by its opposite.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlbm {

enum StoreMode { kF64 = 0, kF32 = 1, kF16Dev = 2 };
enum FieldMode { kFieldNone = 0, kFieldUniform = 1, kFieldMap = 2 };

template <int Q> struct Lat;

template <> struct Lat<9> {
    static constexpr int D = 2;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                 {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
        return t[i][a];
    }
};

template <> struct Lat<19> {
    static constexpr int D = 3;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[19][3] = {{0, 0, 0},   {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                                  {0, 0, 1},   {0, 0, -1}, {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                                  {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                  {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        return t[i][a];
    }
};

template <int Q>
__host__ __device__ constexpr int csq(int i) {
    return Lat<Q>::c(i, 0) * Lat<Q>::c(i, 0) + Lat<Q>::c(i, 1) * Lat<Q>::c(i, 1) +
           Lat<Q>::c(i, 2) * Lat<Q>::c(i, 2);
}

// Per-launch constants, passed by value as a kernel argument.  The host fills
// both the double and the float copies; a kernel reads the copy of its
// compute type.
struct KParams {
    int nx, ny, nz;
    int ncell;
    int Q;
    // collision
    double om, one_m_om;       // omega = Delta t / tau, 1 - omega
    double xi, beta0;          // lattice constant, reference inverse temperature
    double half_xi2;           // xi^2 / 2
    double a1_0, a1_b, a2_0, a2_b, a3, a4, a5;   // Appendix coefficients
    double w[19];              // cubature weights
    double omw[19];            // omega * w_i
    float omwf[19];
    float one_m_omf, a3f, a4f;
    // F16 scaled-deviation codec: a = ref[k][i] + sc[i] * h, sc[i] a power of two
    float ref[4][19];
    float sc[19];
    float inv_sc[19];
    // magnetic field (Sec. 5): uniform rotation of the Bloch vectors, or a
    // per-cell map mu B [3][N] (device) from which each cell's rotation follows
    int field_mode;
    double rot[9];
    const double* bmap;
    // collision variants (Sec. 3.1 isothermal model, Sec. 3.3 positivity): bits kVar*
    int variant;
};

// Collision variants of the step kernels.
enum VariantBits { kVarIso = 1, kVarPos = 2 };

template <int MODE> struct Store;
template <> struct Store<kF64> { using T = double; using C = double; };
template <> struct Store<kF32> { using T = float; using C = float; };
template <> struct Store<kF16Dev> { using T = _Float16; using C = float; };

template <int MODE>
__device__ __forceinline__ typename Store<MODE>::C decode(typename Store<MODE>::T v, int k, int i,
                                                          const KParams& p) {
    if constexpr (MODE == kF16Dev) {
        return p.ref[k][i] + p.sc[i] * static_cast<float>(v);
    } else {
        (void)k; (void)i; (void)p;
        return v;
    }
}

// Round to the storage type: round-to-nearest-even in every mode.  The F16
// scale of each velocity is a power of two, so scaling by it and by its
// inverse is exact and decode(encode(v)) differs from v only by the
// half-precision rounding of the deviation (no systematic gain).
template <int MODE>
__device__ __forceinline__ typename Store<MODE>::T encode(typename Store<MODE>::C v, int k, int i,
                                                          const KParams& p) {
    if constexpr (MODE == kF16Dev) {
        return static_cast<_Float16>((v - p.ref[k][i]) * p.inv_sc[i]);
    } else {
        (void)k; (void)i; (void)p;
        return v;
    }
}

// Compute-type views of the per-velocity constants.
template <typename C> __device__ __forceinline__ C omw_of(const KParams& p, int i);
template <> __device__ __forceinline__ double omw_of<double>(const KParams& p, int i) { return p.omw[i]; }
template <> __device__ __forceinline__ float omw_of<float>(const KParams& p, int i) { return p.omwf[i]; }

template <typename C> __device__ __forceinline__ C cst(double d, float f);
template <> __device__ __forceinline__ double cst<double>(double d, float) { return d; }
template <> __device__ __forceinline__ float cst<float>(double, float f) { return f; }

// Field layout: row-blocked structure of arrays.  Cells are grouped in
// x-rows (row = y + ny * z); each row holds 4 * Q contiguous segments of nx
// values, one per (Pauli component k, velocity i):
//     element (k, i, x, row) at ((row * 4 + k) * Q + i) * nx + x.
// Lanes along x read and write consecutive addresses of one segment, and a
// workgroup's writes fill one contiguous block of its row.
__host__ __device__ __forceinline__ size_t fidx(int Q, int nx, size_t row, int k, int i, int x) {
    return ((row * 4 + static_cast<size_t>(k)) * Q + i) * static_cast<size_t>(nx) + x;
}

// Element x of a field row whose start (one (row, k, i) segment) is the same
// for the whole wave.  The start stays in scalar registers and each lane adds a
// 32-bit byte offset, so an access costs no 64-bit address arithmetic per lane
// (the empty asm keeps the compiler from folding the segments of one cell into
// a per-lane pointer chain).  x must be non-negative and x * sizeof(T) below
// 2^32 (rows hold at most 2^31 cells).  NT: streaming access (the line is not
// kept in the caches), for fields too large to stay in them between passes.
template <bool NT, typename T>
__device__ __forceinline__ T load_row(const T* row, int x) {
    uint64_t a = reinterpret_cast<uint64_t>(row);
    asm volatile("" : "+s"(a));
    const auto* q = reinterpret_cast<const __attribute__((address_space(1))) T*>(
        reinterpret_cast<const __attribute__((address_space(1))) char*>(a) +
        static_cast<unsigned>(x) * static_cast<unsigned>(sizeof(T)));
    if constexpr (NT) return __builtin_nontemporal_load(q);
    else return *q;
}

template <bool NT, typename T>
__device__ __forceinline__ void store_row(T v, T* row, int x) {
    uint64_t a = reinterpret_cast<uint64_t>(row);
    asm volatile("" : "+s"(a));
    auto* q = reinterpret_cast<__attribute__((address_space(1))) T*>(
        reinterpret_cast<__attribute__((address_space(1))) char*>(a) +
        static_cast<unsigned>(x) * static_cast<unsigned>(sizeof(T)));
    if constexpr (NT) __builtin_nontemporal_store(v, q);
    else *q = v;
}

// Periodic source coordinates of a pull: index [c + 1] holds (x - c) mod n.
__device__ __forceinline__ void pull_coords(int x, int n, int stride, int out[3]) {
    out[0] = ((x + 1 == n) ? 0 : x + 1) * stride;   // c = -1
    out[1] = x * stride;                            // c =  0
    out[2] = ((x == 0) ? n - 1 : x - 1) * stride;   // c = +1
}

// Number of double slots per block in the reduction scratch.
constexpr int kRedSlots = 10;
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// Row k of the rotation of the Bloch vector produced by the magnetic-field
// commutator -i [mu sigma.B, W] over one time step (Sec. 5, Eq. sigmaB_comm):
// W -> U W U*, U = exp(-i Delta t sigma.(mu B)), turns every Bloch vector by
// theta = 2 Delta t |mu B| about the unit axis n of B (Rodrigues):
//   R = cos(theta) I + sin(theta) [n]x + (1 - cos(theta)) n n^T.
__device__ __forceinline__ void rotation_row(const double b[3], int k, double r[3]) {
    const double bb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    if (bb == 0.0) {
        r[0] = (k == 0) ? 1.0 : 0.0;
        r[1] = (k == 1) ? 1.0 : 0.0;
        r[2] = (k == 2) ? 1.0 : 0.0;
        return;
    }
    double sn, cs;
    sincos(2.0 * bb, &sn, &cs);
    const double n[3] = {b[0] / bb, b[1] / bb, b[2] / bb};
    // [n]x row k: (0, -n2, n1), (n2, 0, -n0), (-n1, n0, 0)
    const double cx[3][3] = {{0.0, -n[2], n[1]}, {n[2], 0.0, -n[0]}, {-n[1], n[0], 0.0}};
#pragma unroll
    for (int l = 0; l < 3; ++l) r[l] = ((k == l) ? cs : 0.0) + sn * cx[k][l] + (1.0 - cs) * n[k] * n[l];
}

// The whole rotation: R[3 * k + l], Bloch components k, l = 0..2 (x, y, z).
__device__ __forceinline__ void rotation_matrix(const double b[3], double R[9]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) rotation_row(b, k, R + 3 * k);
}

}  // namespace mlbm
