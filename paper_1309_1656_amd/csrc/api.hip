// C ABI of the library (declared and documented in include/mlbm.h).
//
// Host-side work only: argument validation, constants, launch sequencing,
// the private reduction buffer and status codes.  Every numerical step runs
// in the kernels of step.hip, moments.hip, init.hip, adjoint.hip, eigen.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "constants.hpp"
#include "internal.hpp"
#include "mlbm.h"

using namespace mlbm;

struct mlbm_ctx {
    int Q = 0, d = 0, storage = 0, eq_mode = MLBM_EQ_DIRECT;
    bool positivity = false;        // positivity-limited relaxation (mlbm_set_positivity)
    int64_t nx = 0, ny = 0, nz = 0, N = 0;
    double tau = 0.0, beta0 = 0.0;
    HostConst hc{};
    KParams kp{};
    FdParams fp{};
    double f16_scale = 0.0;
    double f16_ref[4][19] = {};
    LaunchCfg launch;               // step launch shape (automatic by default)
    AdjointCfg adj;                 // adjoint launch shape (automatic by default)
    int device = -1;
    double* d_partials = nullptr;   // reduction partials
    size_t partials_cap = 0;        // in doubles
    double* d_result = nullptr;     // 2 kRedSlots finalised values (two chained reductions)
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return MLBM_OK;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(MLBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

int elem_size(int storage) { return storage == MLBM_STORE_F64 ? 8 : (storage == MLBM_STORE_F32 ? 4 : 2); }

int check_handle(mlbm_handle h) {
    if (!h) return fail(MLBM_EINVAL, "null handle");
    return MLBM_OK;
}

// Relaxation parameters into the kernel block.
void set_tau(mlbm_ctx* h, double tau) {
    h->tau = tau;
    KParams& p = h->kp;
    p.om = 1.0 / tau;
    p.one_m_om = 1.0 - p.om;
    p.one_m_omf = static_cast<float>(p.one_m_om);
    for (int i = 0; i < h->Q; ++i) {
        p.omw[i] = p.om * p.w[i];
        p.omwf[i] = static_cast<float>(p.omw[i]);
    }
}

void set_f16(mlbm_ctx* h, const double* ref, double scale) {
    h->f16_scale = scale;
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < h->Q; ++i) {
            h->f16_ref[k][i] = ref[k * h->Q + i];
            h->kp.ref[k][i] = static_cast<float>(ref[k * h->Q + i]);
        }
    // per-velocity scale: the power of two nearest to w_i S (so |h| <= sqrt(2) max|a - R|/(w_i S))
    for (int i = 0; i < h->Q; ++i) {
        const int e = static_cast<int>(std::lround(std::log2(h->kp.w[i] * scale)));
        h->kp.sc[i] = std::ldexp(1.0f, e);
        h->kp.inv_sc[i] = std::ldexp(1.0f, -e);
    }
}

// Private device buffer: at least `need` doubles of partials plus the result row.
int ensure_scratch(mlbm_ctx* h, size_t need) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (h->device >= 0 && dev != h->device)
        return fail(MLBM_EINVAL, "handle first used on device %d, now called on device %d", h->device, dev);
    if (h->d_partials && h->partials_cap >= need) return MLBM_OK;
    if (h->d_partials) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(h->d_partials));
        h->d_partials = nullptr;
    }
    if (!h->d_result) {
        if (hipMalloc(&h->d_result, 2 * kRedSlots * sizeof(double)) != hipSuccess)
            return fail(MLBM_ENOMEM, "cannot allocate %zu bytes of device memory", 2 * kRedSlots * sizeof(double));
    }
    if (hipMalloc(&h->d_partials, need * sizeof(double)) != hipSuccess) {
        h->d_partials = nullptr;
        return fail(MLBM_ENOMEM, "cannot allocate %zu bytes of device memory", need * sizeof(double));
    }
    h->partials_cap = need;
    h->device = dev;
    return MLBM_OK;
}

int red_scratch(mlbm_ctx* h) { return ensure_scratch(h, static_cast<size_t>(kRedBlocks) * kRedSlots); }

// Partials of the adjoint (nb, one per wave or block) and the tail of their two-stage sum.
size_t adjoint_scratch(int nb) {
    return std::max<size_t>(static_cast<size_t>(nb) + kSumChunks, static_cast<size_t>(kRedBlocks) * kRedSlots);
}

// Host copy of the polynomial factor P_i (Eq. WeqAlgo) for the F16DEV reference.
double host_P(const mlbm_ctx* h, int i, const double u[3], double eps) {
    const KParams& p = h->kp;
    const double b = p.beta0 * eps;
    double eu = 0.0, uu = 0.0;
    for (int c = 0; c < 3; ++c) {
        eu += p.xi * (h->Q == 9 ? Lat<9>::c(i, c) : Lat<19>::c(i, c)) * u[c];
        uu += u[c] * u[c];
    }
    const int c2 = h->Q == 9 ? csq<9>(i) : csq<19>(i);
    return p.a1_0 + p.a1_b * b + (p.a2_0 + p.a2_b * b) * p.beta0 * p.half_xi2 * c2 + p.a3 * p.beta0 * eu +
           p.a4 * (p.beta0 * eu) * (p.beta0 * eu) + p.a5 * p.beta0 * 0.5 * uu;
}

int read_result(mlbm_ctx* h, double out[kRedSlots], hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(out, h->d_result, kRedSlots * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MLBM_OK;
}

int check_init_flags(const double r[kRedSlots]) {
    if (r[8] > 0) return fail(MLBM_EDOMAIN, "%.0f cells outside the Fermi-Dirac domain "
                                            "(need tr rho > 0, |r| < tr rho, T > 0, finite values)", r[8]);
    if (r[9] > 0) return fail(MLBM_ENOCONV, "Fermi-Dirac inversion failed in %.0f cells", r[9]);
    return MLBM_OK;
}

// Reduction buffer of mlbm_moments_noalloc: a file-scope device array, so that
// the call allocates nothing.  Every GPU holds its own copy until the process
// ends; host code uses only the address hipGetSymbolAddress returns for the
// current device (the array's name is not a device address in host code).
constexpr size_t kNoAllocDoubles = static_cast<size_t>(kRedBlocks) * kRedSlots;
__device__ __align__(256) double noalloc_scratch[kNoAllocDoubles];
constexpr int kMaxDevices = 64;

// Device address of noalloc_scratch on the current device, looked up once per device.
int noalloc_scratch_ptr(double** out) {
    static std::mutex mu;
    static double* ptrs[kMaxDevices] = {};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MLBM_EINVAL, "device %d outside the supported 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)));
        ptrs[dev] = static_cast<double*>(p);
    }
    *out = ptrs[dev];
    return MLBM_OK;
}

}  // namespace

extern "C" {

const char* mlbm_last_error(void) { return g_err.c_str(); }

int mlbm_create(mlbm_handle* out, int lattice, const int64_t dims[3], double tau, double beta0, int storage) {
    if (!out || !dims) return fail(MLBM_EINVAL, "null argument");
    *out = nullptr;
    if (lattice != MLBM_D2Q9 && lattice != MLBM_D3Q19) return fail(MLBM_EINVAL, "lattice must be 9 or 19");
    if (storage < MLBM_STORE_F64 || storage > MLBM_STORE_F16DEV) return fail(MLBM_EINVAL, "bad storage type");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return fail(MLBM_EINVAL, "dims must be >= 1");
    if (lattice == MLBM_D2Q9 && dims[2] != 1) return fail(MLBM_EINVAL, "D2Q9 needs nz = 1");
    if (dims[1] > 65535 || dims[2] > 65535) return fail(MLBM_EINVAL, "ny and nz must be <= 65535");
    // the kernels address a cell within its row by a 32-bit byte offset
    if (dims[0] > (int64_t{1} << 29)) return fail(MLBM_EINVAL, "nx must be <= 2^29");
    const long double n = static_cast<long double>(dims[0]) * dims[1] * dims[2];
    if (n >= 2147483648.0L) return fail(MLBM_EINVAL, "at most 2^31 - 1 cells");
    if (!(std::isfinite(tau) && tau > 0.5)) return fail(MLBM_EDOMAIN, "tau must be finite and > 1/2 (got %g)", tau);
    if (!(std::isfinite(beta0) && beta0 > 0.0)) return fail(MLBM_EDOMAIN, "beta0 must be finite and > 0 (got %g)", beta0);

    mlbm_ctx* h = new mlbm_ctx();
    h->Q = lattice;
    h->d = lattice == MLBM_D2Q9 ? 2 : 3;
    h->storage = storage;
    h->nx = dims[0];
    h->ny = dims[1];
    h->nz = dims[2];
    h->N = dims[0] * dims[1] * dims[2];
    h->beta0 = beta0;
    h->hc = host_constants(h->d);
    KParams& p = h->kp;
    p.nx = static_cast<int>(h->nx);
    p.ny = static_cast<int>(h->ny);
    p.nz = static_cast<int>(h->nz);
    p.ncell = static_cast<int>(h->N);
    p.Q = h->Q;
    p.xi = h->hc.xi1 / std::sqrt(beta0);
    p.beta0 = beta0;
    p.half_xi2 = 0.5 * p.xi * p.xi;
    p.a1_0 = h->hc.a1_0;
    p.a1_b = h->hc.a1_b;
    p.a2_0 = h->hc.a2_0;
    p.a2_b = h->hc.a2_b;
    p.a3 = h->hc.a3;
    p.a4 = h->hc.a4;
    p.a5 = h->hc.a5;
    p.a3f = static_cast<float>(p.a3);
    p.a4f = static_cast<float>(p.a4);
    for (int i = 0; i < h->Q; ++i) {
        int nz_ = 0;
        for (int c = 0; c < 3; ++c) nz_ += (h->Q == 9 ? Lat<9>::c(i, c) : Lat<19>::c(i, c)) != 0;
        p.w[i] = h->hc.wcls[nz_];
    }
    set_tau(h, tau);
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 19; ++i) p.ref[k][i] = 0.0f;
    for (int i = 0; i < 19; ++i) p.sc[i] = p.inv_sc[i] = 1.0f;
    p.field_mode = kFieldNone;
    p.bmap = nullptr;
    p.variant = 0;
    for (int j = 0; j < 9; ++j) p.rot[j] = (j % 4 == 0) ? 1.0 : 0.0;
    gauss_legendre(kGL, h->fp.gl_x, h->fp.gl_w);
    *out = h;
    return ok();
}

void mlbm_destroy(mlbm_handle h) {
    if (!h) return;
    if (h->d_partials) (void)hipFree(h->d_partials);
    if (h->d_result) (void)hipFree(h->d_result);
    delete h;
}

int mlbm_get_info(mlbm_handle h, mlbm_info* info) {
    if (int e = check_handle(h)) return e;
    if (!info) return fail(MLBM_EINVAL, "null info");
    std::memset(info, 0, sizeof *info);
    info->lattice = h->Q;
    info->d = h->d;
    info->storage = h->storage;
    info->eq_mode = h->eq_mode;
    info->nx = h->nx;
    info->ny = h->ny;
    info->nz = h->nz;
    info->ncell = h->N;
    info->tau = h->tau;
    info->omega = h->kp.om;
    info->beta0 = h->beta0;
    info->xi = h->kp.xi;
    info->a = h->hc.a;
    for (int i = 0; i < h->Q; ++i) {
        info->w[i] = h->kp.w[i];
        for (int c = 0; c < 3; ++c) info->c[i][c] = h->Q == 9 ? Lat<9>::c(i, c) : Lat<19>::c(i, c);
    }
    info->a1_0 = h->kp.a1_0;
    info->a1_b = h->kp.a1_b;
    info->a2_0 = h->kp.a2_0;
    info->a2_b = h->kp.a2_b;
    info->a3 = h->kp.a3;
    info->a4 = h->kp.a4;
    info->a5 = h->kp.a5;
    const LaunchCfg lc = step_launch(static_cast<int>(h->nx), static_cast<int>(h->ny), static_cast<int>(h->nz), h->Q,
                                     h->storage, h->kp.variant, h->kp.field_mode, h->launch);
    info->launch_block_x = lc.bx;
    info->launch_order = lc.order;
    info->launch_blocks_per_cu = lc.cap;
    info->launch_temporal_stores = lc.stores;
    const AdjointCfg ac = adjoint_launch(static_cast<int>(h->nx), static_cast<int>(h->ny), static_cast<int>(h->nz),
                                         h->Q, h->storage, h->kp.field_mode, h->adj);
    info->adjoint_form = ac.form;
    info->adjoint_block_x = ac.form == kAdjChannel ? ac.lc.bx : 0;
    info->adjoint_order = ac.form == kAdjChannel ? ac.lc.order : -1;
    info->adjoint_blocks_per_cu = ac.form == kAdjChannel ? ac.lc.cap : 0;
    info->adjoint_temporal_stores = ac.form == kAdjChannel ? ac.lc.stores : 0;
    info->f16_scale = h->f16_scale;
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < h->Q; ++i) info->f16_ref[k][i] = h->f16_ref[k][i];
    return ok();
}

int mlbm_field_bytes(mlbm_handle h, size_t* bytes) {
    if (int e = check_handle(h)) return e;
    if (!bytes) return fail(MLBM_EINVAL, "null bytes");
    *bytes = static_cast<size_t>(4) * h->Q * static_cast<size_t>(h->N) * elem_size(h->storage);
    return ok();
}

int mlbm_set_tau(mlbm_handle h, double tau) {
    if (int e = check_handle(h)) return e;
    if (!(std::isfinite(tau) && tau > 0.5)) return fail(MLBM_EDOMAIN, "tau must be finite and > 1/2 (got %g)", tau);
    set_tau(h, tau);
    return ok();
}

static void update_variant(mlbm_handle h) {
    h->kp.variant = (h->eq_mode == MLBM_EQ_ISOTHERMAL ? kVarIso : 0) | (h->positivity ? kVarPos : 0);
}

int mlbm_set_eq_mode(mlbm_handle h, int mode) {
    if (int e = check_handle(h)) return e;
    if (mode != MLBM_EQ_DIRECT && mode != MLBM_EQ_EIGEN && mode != MLBM_EQ_ISOTHERMAL)
        return fail(MLBM_EINVAL, "bad equilibrium mode");
    if (mode == MLBM_EQ_EIGEN && h->storage != MLBM_STORE_F64)
        return fail(MLBM_EINVAL, "the eigen-channel mode needs double storage");
    if (mode == MLBM_EQ_EIGEN && h->positivity)
        return fail(MLBM_EINVAL, "the eigen-channel mode does not take the positivity limit");
    if (mode != MLBM_EQ_DIRECT && h->kp.field_mode != kFieldNone)
        return fail(MLBM_EINVAL, "the magnetic field needs the direct equilibrium mode");
    h->eq_mode = mode;
    update_variant(h);
    return ok();
}

int mlbm_set_positivity(mlbm_handle h, int on) {
    if (int e = check_handle(h)) return e;
    if (on != 0 && on != 1) return fail(MLBM_EINVAL, "positivity flag must be 0 or 1");
    if (on && h->eq_mode == MLBM_EQ_EIGEN)
        return fail(MLBM_EINVAL, "the eigen-channel mode does not take the positivity limit");
    if (on && h->kp.field_mode != kFieldNone)
        return fail(MLBM_EINVAL, "the positivity limit does not take a magnetic field");
    h->positivity = on != 0;
    update_variant(h);
    return ok();
}

int mlbm_set_magnetic_field(mlbm_handle h, const double mu_b[3]) {
    if (int e = check_handle(h)) return e;
    const bool off = !mu_b || (mu_b[0] == 0.0 && mu_b[1] == 0.0 && mu_b[2] == 0.0);
    if (!off) {
        if (!(std::isfinite(mu_b[0]) && std::isfinite(mu_b[1]) && std::isfinite(mu_b[2])))
            return fail(MLBM_EINVAL, "non-finite magnetic field");
        if (h->eq_mode != MLBM_EQ_DIRECT || h->positivity)
            return fail(MLBM_EINVAL, "the magnetic field needs the direct equilibrium mode without the positivity limit");
    }
    KParams& p = h->kp;
    p.bmap = nullptr;
    if (off) {
        p.field_mode = kFieldNone;
        for (int j = 0; j < 9; ++j) p.rot[j] = (j % 4 == 0) ? 1.0 : 0.0;
        return ok();
    }
    // rotation by theta = 2 dt |mu B| about n = B / |B| (Rodrigues), dt = 1
    const double bb = std::sqrt(mu_b[0] * mu_b[0] + mu_b[1] * mu_b[1] + mu_b[2] * mu_b[2]);
    const double n[3] = {mu_b[0] / bb, mu_b[1] / bb, mu_b[2] / bb};
    const double cs = std::cos(2.0 * bb), sn = std::sin(2.0 * bb);
    const double cx[3][3] = {{0.0, -n[2], n[1]}, {n[2], 0.0, -n[0]}, {-n[1], n[0], 0.0}};
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) p.rot[k * 3 + l] = (k == l ? cs : 0.0) + sn * cx[k][l] + (1.0 - cs) * n[k] * n[l];
    p.field_mode = kFieldUniform;
    return ok();
}

int mlbm_set_magnetic_field_map(mlbm_handle h, const double* mu_b) {
    if (int e = check_handle(h)) return e;
    if (mu_b && (h->eq_mode != MLBM_EQ_DIRECT || h->positivity))
        return fail(MLBM_EINVAL, "the magnetic field needs the direct equilibrium mode without the positivity limit");
    h->kp.bmap = mu_b;
    h->kp.field_mode = mu_b ? kFieldMap : kFieldNone;
    return ok();
}

int mlbm_set_launch(mlbm_handle h, int block_x, int order, int blocks_per_cu) {
    if (int e = check_handle(h)) return e;
    if (block_x != 0 && block_x != 64 && block_x != 128) return fail(MLBM_EINVAL, "block_x must be 0, 64 or 128");
    if (order < -1 || order > 2) return fail(MLBM_EINVAL, "order must be -1, 0, 1 or 2");
    if (blocks_per_cu < -1 || blocks_per_cu > 32) return fail(MLBM_EINVAL, "blocks_per_cu must be in [-1, 32]");
    h->launch.bx = block_x;
    h->launch.order = order;
    h->launch.cap = blocks_per_cu;
    return ok();
}

int mlbm_set_adjoint_launch(mlbm_handle h, int form, int block_x, int order, int blocks_per_cu, int stores) {
    if (int e = check_handle(h)) return e;
    if (form < MLBM_ADJ_AUTO || form > MLBM_ADJ_CELL) return fail(MLBM_EINVAL, "form must be 0, 1 or 2");
    if (block_x != 0 && block_x != 64 && block_x != 128) return fail(MLBM_EINVAL, "block_x must be 0, 64 or 128");
    if (order < -1 || order > 2) return fail(MLBM_EINVAL, "order must be -1, 0, 1 or 2");
    if (blocks_per_cu < -1 || blocks_per_cu > 32) return fail(MLBM_EINVAL, "blocks_per_cu must be in [-1, 32]");
    if (stores < -1 || stores > 1) return fail(MLBM_EINVAL, "store policy must be -1, 0 or 1");
    h->adj.form = form;
    h->adj.lc.bx = block_x;
    h->adj.lc.order = order;
    h->adj.lc.cap = blocks_per_cu;
    h->adj.lc.stores = stores;
    return ok();
}

int mlbm_set_store_policy(mlbm_handle h, int policy) {
    if (int e = check_handle(h)) return e;
    if (policy < -1 || policy > 1) return fail(MLBM_EINVAL, "store policy must be -1, 0 or 1");
    h->launch.stores = policy;
    return ok();
}

int mlbm_set_f16_reference(mlbm_handle h, const double* ref, double scale) {
    if (int e = check_handle(h)) return e;
    if (h->storage != MLBM_STORE_F16DEV) return fail(MLBM_EINVAL, "handle does not use F16DEV storage");
    if (!ref) return fail(MLBM_EINVAL, "null reference");
    if (!(std::isfinite(scale) && scale > 0.0)) return fail(MLBM_EINVAL, "scale must be finite and > 0");
    for (int j = 0; j < 4 * h->Q; ++j)
        if (!std::isfinite(ref[j])) return fail(MLBM_EINVAL, "non-finite reference value");
    set_f16(h, ref, scale);
    return ok();
}

// The three init phases shared by both ways of naming the state; `a` is rho4
// (kFromDensity) or nu2 (kFromChemical).
static int init_state(mlbm_handle h, int src, void* W, const double* a, const double* axis, const double* u,
                      const double* T, void* stream) {
    if (int e = red_scratch(h)) return e;
    hipStream_t s = as_stream(stream);
    double r[kRedSlots];
    if (h->storage == MLBM_STORE_F16DEV) {
        // global means of the initial state (Eqs. GlobalDensity, GlobalVelocity, GlobalTotalEnergy)
        HIP_TRY(launch_init(h->Q, h->storage, 0, src, W, a, axis, u, T, h->kp, h->fp, h->d_partials, s));
        HIP_TRY(launch_finalize(h->d_partials, kRedBlocks, kRedSlots, 0u, h->d_result, nullptr, 1.0, s));
        if (int e = read_result(h, r, s)) return e;
        if (int e = check_init_flags(r)) return e;
        const double invN = 1.0 / static_cast<double>(h->N);
        double rbar[4], ubar[3], uu = 0.0;
        for (int k = 0; k < 4; ++k) rbar[k] = r[k] * invN;
        for (int c = 0; c < 3; ++c) {
            ubar[c] = r[4 + c] * invN / rbar[0];
            uu += ubar[c] * ubar[c];
        }
        const double epsbar = r[7] * invN / rbar[0] - 0.5 * uu;
        double ref[4 * 19];
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < h->Q; ++i) ref[k * h->Q + i] = h->kp.w[i] * rbar[k] * host_P(h, i, ubar, epsbar);
        set_f16(h, ref, 1.0);
        // largest scaled deviation max |a - R| / w_i fixes the power-of-two scale
        HIP_TRY(launch_init(h->Q, h->storage, 1, src, W, a, axis, u, T, h->kp, h->fp, h->d_partials, s));
        HIP_TRY(launch_finalize(h->d_partials, kRedBlocks, kRedSlots, 1u, h->d_result, nullptr, 1.0, s));
        if (int e = read_result(h, r, s)) return e;
        if (int e = check_init_flags(r)) return e;
        double scale = 1.0;
        if (r[0] > 0.0) {
            int ex = 0;
            const double m = std::frexp(r[0], &ex);   // r0 = m 2^ex, m in [0.5, 1)
            scale = std::ldexp(1.0, m == 0.5 ? ex - 1 : ex);
        }
        set_f16(h, ref, scale);
    }
    HIP_TRY(launch_init(h->Q, h->storage, 2, src, W, a, axis, u, T, h->kp, h->fp, h->d_partials, s));
    HIP_TRY(launch_finalize(h->d_partials, kRedBlocks, kRedSlots, 0u, h->d_result, nullptr, 1.0, s));
    if (int e = read_result(h, r, s)) return e;
    if (int e = check_init_flags(r)) return e;
    return ok();
}

int mlbm_init_equilibrium(mlbm_handle h, void* W, const double* rho4, const double* u, const double* T,
                          void* stream) {
    if (int e = check_handle(h)) return e;
    if (!W || !rho4 || !u || !T) return fail(MLBM_EINVAL, "null argument");
    return init_state(h, kFromDensity, W, rho4, nullptr, u, T, stream);
}

int mlbm_init_chemical(mlbm_handle h, void* W, const double* nu, const double* axis, const double* u, const double* T,
                       void* stream) {
    if (int e = check_handle(h)) return e;
    if (!W || !nu || !u || !T) return fail(MLBM_EINVAL, "null argument");
    return init_state(h, kFromChemical, W, nu, axis, u, T, stream);
}

int mlbm_step(mlbm_handle h, void* W, void* scratch, int nsteps, void* stream) {
    if (int e = check_handle(h)) return e;
    if (!W || !scratch) return fail(MLBM_EINVAL, "null field");
    if (W == scratch) return fail(MLBM_EINVAL, "W and scratch must be distinct");
    if (nsteps < 0) return fail(MLBM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return ok();
    hipStream_t s = as_stream(stream);
    const bool eig = h->eq_mode == MLBM_EQ_EIGEN;
    auto run = [&](StepKind kind, const void* a, void* b) -> hipError_t {
        if (eig && kind != StepKind::StreamOnly) return launch_step_eigen(kind, h->Q, a, b, h->kp, h->fp, nullptr, s);
        return launch_step(kind, h->Q, h->storage, a, b, h->kp, h->fp, h->launch, s);
    };
    if (nsteps == 1 || eig) {
        // After the collide-only pass and nsteps - 1 fused passes the
        // post-collision state sits in `scratch`; the stream-only pass then
        // returns the pre-collision state to W.
        void* cur = (nsteps % 2 == 0) ? W : scratch;
        void* other = (cur == W) ? scratch : W;
        HIP_TRY(run(StepKind::CollideOnly, W, cur));
        for (int j = 1; j < nsteps; ++j) {
            HIP_TRY(run(StepKind::Fused, cur, other));
            std::swap(cur, other);
        }
        HIP_TRY(run(StepKind::StreamOnly, cur, W));
        return ok();
    }
    // nsteps passes: the collide-only pass, nsteps - 2 fused passes, and a last
    // fused pass whose collided values go where the final streaming sends them,
    // straight into W.  The state before that last pass is left in `scratch`.
    void* cur = (nsteps % 2 == 0) ? scratch : W;
    void* other = (cur == W) ? scratch : W;
    HIP_TRY(run(StepKind::CollideOnly, W, cur));
    for (int j = 1; j < nsteps - 1; ++j) {
        HIP_TRY(run(StepKind::Fused, cur, other));
        std::swap(cur, other);
    }
    HIP_TRY(run(StepKind::FusedPush, cur, W));
    return ok();
}

int mlbm_step_states(mlbm_handle h, const void* src, void* dst, void* states, int nstates, int nsteps,
                     void* stream) {
    if (int e = check_handle(h)) return e;
    if (!src || !dst) return fail(MLBM_EINVAL, "null field");
    if (nsteps < 0) return fail(MLBM_EINVAL, "nsteps must be >= 0");
    if (src == dst) return fail(MLBM_EINVAL, "src and dst must be distinct");
    size_t fb = 0;
    mlbm_field_bytes(h, &fb);
    hipStream_t s = as_stream(stream);
    if (nsteps == 0) {
        HIP_TRY(hipMemcpyAsync(dst, src, fb, hipMemcpyDeviceToDevice, s));
        return ok();
    }
    if (!states) return fail(MLBM_EINVAL, "null states");
    if (nstates < 1 || (nsteps > 1 && nstates < 2))
        return fail(MLBM_EINVAL, "need nstates >= 1, and >= 2 for more than one step (got %d)", nstates);
    const uintptr_t a = reinterpret_cast<uintptr_t>(states), end = a + static_cast<uintptr_t>(nstates) * fb;
    auto inside = [&](const void* q) {
        const uintptr_t u = reinterpret_cast<uintptr_t>(q);
        return u + fb > a && u < end;
    };
    if (inside(src) || inside(dst)) return fail(MLBM_EINVAL, "src and dst must not overlap the states");
    const bool eig = h->eq_mode == MLBM_EQ_EIGEN;
    auto run = [&](StepKind kind, const void* x, void* y) -> hipError_t {
        if (eig && kind != StepKind::StreamOnly) return launch_step_eigen(kind, h->Q, x, y, h->kp, h->fp, nullptr, s);
        return launch_step(kind, h->Q, h->storage, x, y, h->kp, h->fp, h->launch, s);
    };
    char* st = static_cast<char*>(states);
    auto slot = [&](int j) { return st + static_cast<size_t>(j % nstates) * fb; };
    HIP_TRY(run(StepKind::CollideOnly, src, slot(0)));
    for (int j = 1; j < nsteps; ++j) HIP_TRY(run(StepKind::Fused, slot(j - 1), slot(j)));
    HIP_TRY(run(StepKind::StreamOnly, slot(nsteps - 1), dst));
    return ok();
}

int mlbm_collide(mlbm_handle h, const void* src, void* dst, void* stream) {
    if (int e = check_handle(h)) return e;
    if (!src || !dst) return fail(MLBM_EINVAL, "null field");
    hipStream_t s = as_stream(stream);
    if (h->eq_mode == MLBM_EQ_EIGEN) HIP_TRY(launch_step_eigen(StepKind::CollideOnly, h->Q, src, dst, h->kp, h->fp, nullptr, s));
    else HIP_TRY(launch_step(StepKind::CollideOnly, h->Q, h->storage, src, dst, h->kp, h->fp, h->launch, s));
    return ok();
}

int mlbm_stream(mlbm_handle h, const void* src, void* dst, void* stream) {
    if (int e = check_handle(h)) return e;
    if (!src || !dst) return fail(MLBM_EINVAL, "null field");
    if (src == dst) return fail(MLBM_EINVAL, "streaming needs distinct src and dst");
    HIP_TRY(launch_step(StepKind::StreamOnly, h->Q, h->storage, src, dst, h->kp, h->fp, h->launch, as_stream(stream)));
    return ok();
}

int mlbm_moments(mlbm_handle h, const void* W, double* rho4, double* u, double* eps, double* global8,
                 int64_t* n_neg_eig, void* stream) {
    if (int e = check_handle(h)) return e;
    if (!W) return fail(MLBM_EINVAL, "null field");
    if (int e = red_scratch(h)) return e;
    hipStream_t s = as_stream(stream);
    HIP_TRY(launch_moments(h->Q, h->storage, W, rho4, u, eps, h->kp, h->d_partials, s));
    if (!global8 && !n_neg_eig) return ok();
    HIP_TRY(launch_finalize(h->d_partials, kRedBlocks, kRedSlots, 0u, h->d_result, nullptr, 1.0, s));
    double r[kRedSlots];
    if (int e = read_result(h, r, s)) return e;
    if (global8) {
        const double invN = 1.0 / static_cast<double>(h->N);
        for (int k = 0; k < 8; ++k) global8[k] = r[k] * invN;
    }
    if (n_neg_eig) *n_neg_eig = static_cast<int64_t>(r[8]);
    if (r[9] > 0) return fail(MLBM_ENONFINITE, "%.0f non-finite values in the field", r[9]);
    return ok();
}

int mlbm_moments_noalloc(mlbm_handle h, const void* W, double* rho4, double* u, double* eps, double* sums,
                         void* stream) {
    if (int e = check_handle(h)) return e;
    if (!W) return fail(MLBM_EINVAL, "null field");
    // the reduction uses a fixed grid of kRedBlocks blocks, whatever the lattice size
    static_assert(static_cast<size_t>(kRedBlocks) * kRedSlots <= kNoAllocDoubles, "reduction buffer too small");
    double* scratch = nullptr;
    if (int e = noalloc_scratch_ptr(&scratch)) return e;
    hipStream_t s = as_stream(stream);
    HIP_TRY(launch_moments(h->Q, h->storage, W, rho4, u, eps, h->kp, scratch, s));
    if (sums) HIP_TRY(launch_finalize(scratch, kRedBlocks, kRedSlots, 0u, sums, nullptr, 1.0, s));
    return ok();
}

int mlbm_relaxation(mlbm_handle h, const void* W, double out[8], void* stream) {
    if (int e = check_handle(h)) return e;
    if (!W || !out) return fail(MLBM_EINVAL, "null argument");
    if (int e = red_scratch(h)) return e;
    hipStream_t s = as_stream(stream);
    // pass 1: global sums into d_result[0..); pass 2 reads them on the device
    HIP_TRY(launch_moments(h->Q, h->storage, W, nullptr, nullptr, nullptr, h->kp, h->d_partials, s));
    HIP_TRY(launch_finalize(h->d_partials, kRedBlocks, kRedSlots, 0u, h->d_result, nullptr, 1.0, s));
    HIP_TRY(launch_relaxation(h->Q, h->storage, W, h->d_result, h->kp, h->d_partials, s));
    HIP_TRY(launch_finalize(h->d_partials, kRedBlocks, kRedSlots, 7u, h->d_result + kRedSlots, nullptr, 1.0, s));
    double r[2 * kRedSlots];
    HIP_TRY(hipMemcpyAsync(r, h->d_result, 2 * kRedSlots * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (r[9] > 0) return fail(MLBM_ENONFINITE, "%.0f non-finite values in the field", r[9]);
    const double* q = r + kRedSlots;
    const double invN = 1.0 / static_cast<double>(h->N);
    out[0] = q[0];
    out[1] = q[1];
    out[2] = q[2];
    out[3] = q[3] * invN;
    out[4] = q[4] * invN;
    for (int j = 5; j < 8; ++j) out[j] = std::sqrt(q[j] * invN);
    return ok();
}

int mlbm_spin_loss(mlbm_handle h, const void* W, const double* r_target, double* loss, void* lam, void* stream) {
    if (int e = check_handle(h)) return e;
    if (!W || !r_target) return fail(MLBM_EINVAL, "null argument");
    if (h->storage == MLBM_STORE_F16DEV) return fail(MLBM_EINVAL, "the spin loss needs F64 or F32 storage");
    if (lam && lam == W) return fail(MLBM_EINVAL, "lam must not alias W");
    if (int e = red_scratch(h)) return e;
    hipStream_t s = as_stream(stream);
    HIP_TRY(launch_spin_loss(h->Q, h->storage, W, r_target, lam, h->kp, h->d_partials, s));
    if (loss) {
        HIP_TRY(launch_finalize(h->d_partials, kRedBlocks, kRedSlots, 0u, h->d_result, nullptr,
                                1.0 / static_cast<double>(h->N), s));
        HIP_TRY(hipMemcpyAsync(loss, h->d_result, sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    return ok();
}

int mlbm_adjoint_step(mlbm_handle h, const void* W_n, const void* lam_next, void* lam_n, double* dL_domega,
                      void* stream) {
    if (int e = check_handle(h)) return e;
    if (!W_n || !lam_next || !lam_n) return fail(MLBM_EINVAL, "null field");
    if (h->storage == MLBM_STORE_F16DEV) return fail(MLBM_EINVAL, "the adjoint needs F64 or F32 storage");
    if (h->eq_mode != MLBM_EQ_DIRECT || h->positivity)
        return fail(MLBM_EINVAL, "the adjoint needs the direct equilibrium mode without the positivity limit");
    if (lam_n == W_n || lam_n == lam_next) return fail(MLBM_EINVAL, "lam_n must not alias the inputs");
    const int nb = adjoint_blocks(h->kp, h->storage, h->adj);
    if (int e = ensure_scratch(h, adjoint_scratch(nb))) return e;
    hipStream_t s = as_stream(stream);
    HIP_TRY(launch_adjoint(h->Q, h->storage, false, W_n, lam_next, lam_n, h->kp, h->d_partials, false, h->adj, s));
    if (dL_domega) HIP_TRY(launch_sum_into(h->d_partials, nb, h->d_partials + nb, dL_domega, 1.0, s));
    return ok();
}

// Checks shared by mlbm_adjoint_segment and mlbm_adjoint_sweep; also sizes the partials.
static int adjoint_checks(mlbm_handle h, const void* W, const void* states, int nsteps, void* lam, void* lam_tmp) {
    if (int e = check_handle(h)) return e;
    if (!W || !lam || !lam_tmp || (nsteps > 1 && !states)) return fail(MLBM_EINVAL, "null field");
    if (nsteps < 0) return fail(MLBM_EINVAL, "nsteps must be >= 0");
    if (h->storage == MLBM_STORE_F16DEV) return fail(MLBM_EINVAL, "the adjoint needs F64 or F32 storage");
    if (h->eq_mode != MLBM_EQ_DIRECT || h->positivity)
        return fail(MLBM_EINVAL, "the adjoint needs the direct equilibrium mode without the positivity limit");
    if (lam == lam_tmp || lam == W || lam_tmp == W) return fail(MLBM_EINVAL, "lam, lam_tmp and W must be distinct");
    if (nsteps == 0) return MLBM_OK;
    const int nb = adjoint_blocks(h->kp, h->storage, h->adj);
    return ensure_scratch(h, adjoint_scratch(nb));
}

// Reverse sweep over nsteps adjoint steps: step j reads W_j, gathered from
// states[j - 1] (post-collision) for j >= 1 and W itself for j = 0.
// With w_post, W is the post-collision state of the step before the segment and
// step 0 gathers its state from W by a pull as well.
static int adjoint_reverse(mlbm_handle h, const void* W, bool w_post, const char* st, int nsteps, void* lam,
                           void* lam_tmp, double* dL_domega, hipStream_t s) {
    const int nb = adjoint_blocks(h->kp, h->storage, h->adj);
    size_t fb = 0;
    mlbm_field_bytes(h, &fb);
    void* in = lam;
    void* out = lam_tmp;
    for (int j = nsteps - 1; j >= 0; --j) {
        const bool pulled = j > 0 || w_post;
        const void* wsrc = j > 0 ? static_cast<const void*>(st + (j - 1) * fb) : W;
        // block partials of dL/domega accumulate over the sweep: one final sum
        HIP_TRY(launch_adjoint(h->Q, h->storage, pulled, wsrc, in, out, h->kp, h->d_partials, j < nsteps - 1, h->adj, s));
        void* t = in;
        in = out;
        out = t;
    }
    if (dL_domega) HIP_TRY(launch_sum_into(h->d_partials, nb, h->d_partials + nb, dL_domega, 1.0, s));
    if (in != lam) HIP_TRY(hipMemcpyAsync(lam, in, fb, hipMemcpyDeviceToDevice, s));
    return ok();
}

int mlbm_adjoint_segment(mlbm_handle h, const void* W, void* states, int nsteps, void* lam, void* lam_tmp,
                         double* dL_domega, void* stream) {
    if (int e = adjoint_checks(h, W, states, nsteps, lam, lam_tmp)) return e;
    if (nsteps == 0) return ok();
    hipStream_t s = as_stream(stream);
    size_t fb = 0;
    mlbm_field_bytes(h, &fb);
    char* st = static_cast<char*>(states);
    // forward recomputation: states[j] = post-collision state of step j (j = 0 .. nsteps - 2)
    if (nsteps > 1) HIP_TRY(launch_step(StepKind::CollideOnly, h->Q, h->storage, W, st, h->kp, h->fp, h->launch, s));
    for (int j = 1; j < nsteps - 1; ++j)
        HIP_TRY(launch_step(StepKind::Fused, h->Q, h->storage, st + (j - 1) * fb, st + j * fb, h->kp, h->fp, h->launch, s));
    return adjoint_reverse(h, W, false, st, nsteps, lam, lam_tmp, dL_domega, s);
}

int mlbm_adjoint_sweep(mlbm_handle h, const void* W, const void* states, int nsteps, void* lam, void* lam_tmp,
                       double* dL_domega, void* stream) {
    if (int e = adjoint_checks(h, W, states, nsteps, lam, lam_tmp)) return e;
    if (nsteps == 0) return ok();
    return adjoint_reverse(h, W, false, static_cast<const char*>(states), nsteps, lam, lam_tmp, dL_domega,
                           as_stream(stream));
}

int mlbm_adjoint_sweep_post(mlbm_handle h, const void* S_prev, const void* states, int nsteps, void* lam,
                            void* lam_tmp, double* dL_domega, void* stream) {
    if (int e = adjoint_checks(h, S_prev, states, nsteps, lam, lam_tmp)) return e;
    if (nsteps == 0) return ok();
    return adjoint_reverse(h, S_prev, true, static_cast<const char*>(states), nsteps, lam, lam_tmp, dL_domega,
                           as_stream(stream));
}

int mlbm_step_post(mlbm_handle h, const void* src, int src_post, void* dst, void* states, int nstates, int nsteps,
                   void* stream) {
    if (int e = check_handle(h)) return e;
    if (!src) return fail(MLBM_EINVAL, "null src");
    if (src_post != 0 && src_post != 1) return fail(MLBM_EINVAL, "src_post must be 0 or 1");
    if (nsteps < 0) return fail(MLBM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return ok();
    if (h->eq_mode == MLBM_EQ_EIGEN) return fail(MLBM_EINVAL, "mlbm_step_post does not take the eigen-channel mode");
    // states written to `states`: all but the last one when dst is given
    const int m = dst ? nsteps - 1 : nsteps;
    if (m > 0 && (!states || nstates < 1)) return fail(MLBM_EINVAL, "need states with nstates >= 1");
    if (m > 1 && nstates < 2) return fail(MLBM_EINVAL, "need nstates >= 2 for more than one kept state (got %d)", nstates);
    size_t fb = 0;
    mlbm_field_bytes(h, &fb);
    const uintptr_t a = reinterpret_cast<uintptr_t>(states);
    const uintptr_t end = m > 0 ? a + static_cast<uintptr_t>(std::min(m, nstates)) * fb : a;
    auto in_states = [&](const void* q) {
        const uintptr_t u = reinterpret_cast<uintptr_t>(q);
        return m > 0 && u + fb > a && u < end;
    };
    auto overlap = [&](const void* p1, const void* p2) {
        const uintptr_t u = reinterpret_cast<uintptr_t>(p1), v = reinterpret_cast<uintptr_t>(p2);
        return u < v + fb && v < u + fb;
    };
    if (in_states(src)) return fail(MLBM_EINVAL, "src must not overlap the states written");
    if (dst && (in_states(dst) || overlap(dst, src))) return fail(MLBM_EINVAL, "dst must not overlap src or the states written");
    hipStream_t s = as_stream(stream);
    char* st = static_cast<char*>(states);
    auto out = [&](int j) -> void* { return (dst && j == nsteps - 1) ? dst : st + static_cast<size_t>(j % nstates) * fb; };
    HIP_TRY(launch_step(src_post ? StepKind::Fused : StepKind::CollideOnly, h->Q, h->storage, src, out(0), h->kp, h->fp,
                        h->launch, s));
    for (int j = 1; j < nsteps; ++j)
        HIP_TRY(launch_step(StepKind::Fused, h->Q, h->storage, out(j - 1), out(j), h->kp, h->fp, h->launch, s));
    return ok();
}

int mlbm_device_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst) return fail(MLBM_EINVAL, "null pointer");
    if (bytes % 16 != 0) return fail(MLBM_EINVAL, "bytes must be a multiple of 16 (got %zu)", bytes);
    const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
    if (a % 16 != 0 || b % 16 != 0) return fail(MLBM_EINVAL, "src and dst must be 16-byte aligned");
    if (a < b + bytes && b < a + bytes && bytes > 0) return fail(MLBM_EINVAL, "src and dst overlap");
    // one thread per 16 bytes and at most 2^31 threads in the grid
    if (bytes > (static_cast<size_t>(1) << 35)) return fail(MLBM_EINVAL, "at most 2^35 bytes per call");
    HIP_TRY(launch_copy16(src, dst, bytes / 16, as_stream(stream)));
    return ok();
}

}  // extern "C"
