/*
 * A plain C client of libmlbm.so: no Python, no torch.  Creates a D3Q19
 * handle, fills the macroscopic inputs on the host, copies them to device
 * memory obtained with hipMalloc, builds the Fermi-Dirac initial state, takes
 * a few steps and prints the global averages before and after (Eqs.
 * GlobalDensity, GlobalVelocity, GlobalTotalEnergy) with 17 digits, one
 * line each.  Usage: mlbm_c_demo nx ny nz nsteps.  Exit status 0 on success.
 * The inputs are the deterministic fields below, repeated by the test that
 * runs this program.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "mlbm.h"

#define CHECK(call)                                                                   \
    do {                                                                              \
        int st_ = (call);                                                             \
        if (st_ != MLBM_OK) {                                                         \
            fprintf(stderr, "%s failed: %d %s\n", #call, st_, mlbm_last_error());     \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

#define HIPCHECK(call)                                                                \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));         \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 5) {
        fprintf(stderr, "usage: %s nx ny nz nsteps\n", argv[0]);
        return 2;
    }
    const int64_t dims[3] = {atoll(argv[1]), atoll(argv[2]), atoll(argv[3])};
    const int nsteps = atoi(argv[4]);
    const double pi = 3.14159265358979323846;
    mlbm_handle h = NULL;
    CHECK(mlbm_create(&h, MLBM_D3Q19, dims, 0.8, 1.0, MLBM_STORE_F64));
    mlbm_info info;
    CHECK(mlbm_get_info(h, &info));
    const size_t N = (size_t)info.ncell;
    double* host = (double*)malloc(8 * N * sizeof(double));   /* rho4 (4), u (3), T (1) */
    if (!host) return 1;
    for (int64_t z = 0; z < dims[2]; ++z)
        for (int64_t y = 0; y < dims[1]; ++y)
            for (int64_t x = 0; x < dims[0]; ++x) {
                const size_t n = (size_t)(x + dims[0] * (y + dims[1] * z));
                const double sx = 2.0 * pi * (double)x / (double)dims[0];
                const double sy = 2.0 * pi * (double)y / (double)dims[1];
                const double sz = 2.0 * pi * (double)z / (double)dims[2];
                host[0 * N + n] = 1.0 + 0.05 * sin(sx) * cos(sy);
                host[1 * N + n] = 0.1 * sin(sz);
                host[2 * N + n] = 0.05;
                host[3 * N + n] = 0.1 * cos(sx);
                host[4 * N + n] = info.xi * 0.02 * sin(sy);
                host[5 * N + n] = info.xi * 0.02 * cos(sz);
                host[6 * N + n] = info.xi * 0.02 * sin(sx);
                host[7 * N + n] = 1.0 + 0.02 * cos(sx + sy + sz);
            }
    size_t fb = 0;
    CHECK(mlbm_field_bytes(h, &fb));
    double* d_in = NULL;
    void *W = NULL, *scratch = NULL;
    HIPCHECK(hipMalloc((void**)&d_in, 8 * N * sizeof(double)));
    HIPCHECK(hipMalloc(&W, fb));
    HIPCHECK(hipMalloc(&scratch, fb));
    HIPCHECK(hipMemcpy(d_in, host, 8 * N * sizeof(double), hipMemcpyHostToDevice));
    CHECK(mlbm_init_equilibrium(h, W, d_in, d_in + 4 * N, d_in + 7 * N, NULL));
    double g[8];
    int64_t nneg = -1;
    CHECK(mlbm_moments(h, W, NULL, NULL, NULL, g, &nneg, NULL));
    printf("global0");
    for (int k = 0; k < 8; ++k) printf(" %.17g", g[k]);
    printf("\n");
    CHECK(mlbm_step(h, W, scratch, nsteps, NULL));
    CHECK(mlbm_moments(h, W, NULL, NULL, NULL, g, &nneg, NULL));
    printf("global1");
    for (int k = 0; k < 8; ++k) printf(" %.17g", g[k]);
    printf("\nnneg %lld\n", (long long)nneg);
    HIPCHECK(hipFree(d_in));
    HIPCHECK(hipFree(W));
    HIPCHECK(hipFree(scratch));
    mlbm_destroy(h);
    free(host);
    return 0;
}
