/*
 * Host-only exercise of the C ABI for the sanitizer build (AddressSanitizer
 * and UndefinedBehaviorSanitizer on the host code of the library and of this
 * program).  Every call here returns before any device work: handle
 * creation and destruction, info, field sizes, every setter with good and bad
 * arguments, and the argument checks of the compute entry points.  Exit
 * status 0 when every status code is the expected one.
 */
#include <stdio.h>
#include <string.h>

#include "mlbm.h"

static int failures = 0;

#define EXPECT(call, want)                                                                  \
    do {                                                                                    \
        int got_ = (call);                                                                  \
        if (got_ != (want)) {                                                               \
            fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, \
                    got_, (want), mlbm_last_error());                                       \
            ++failures;                                                                     \
        }                                                                                   \
    } while (0)

int main(void) {
    const int64_t dims3[3] = {13, 9, 11}, dims2[3] = {37, 70, 1}, bad2[3] = {8, 8, 2}, zero[3] = {0, 8, 8};
    mlbm_handle h = NULL, h2 = NULL, h16 = NULL;
    EXPECT(mlbm_create(&h, MLBM_D3Q19, dims3, 0.8, 1.0, MLBM_STORE_F64), MLBM_OK);
    EXPECT(mlbm_create(&h2, MLBM_D2Q9, dims2, 0.6, 1.2, MLBM_STORE_F32), MLBM_OK);
    EXPECT(mlbm_create(&h16, MLBM_D3Q19, dims3, 0.8, 1.0, MLBM_STORE_F16DEV), MLBM_OK);
    mlbm_handle bad = NULL;
    EXPECT(mlbm_create(&bad, 10, dims3, 0.8, 1.0, MLBM_STORE_F64), MLBM_EINVAL);
    EXPECT(mlbm_create(&bad, MLBM_D2Q9, bad2, 0.8, 1.0, MLBM_STORE_F64), MLBM_EINVAL);
    EXPECT(mlbm_create(&bad, MLBM_D3Q19, zero, 0.8, 1.0, MLBM_STORE_F64), MLBM_EINVAL);
    EXPECT(mlbm_create(&bad, MLBM_D3Q19, dims3, 0.5, 1.0, MLBM_STORE_F64), MLBM_EDOMAIN);
    EXPECT(mlbm_create(&bad, MLBM_D3Q19, dims3, 0.8, -1.0, MLBM_STORE_F64), MLBM_EDOMAIN);
    EXPECT(mlbm_create(NULL, MLBM_D3Q19, dims3, 0.8, 1.0, MLBM_STORE_F64), MLBM_EINVAL);
    if (strlen(mlbm_last_error()) == 0) ++failures;

    mlbm_info info;
    EXPECT(mlbm_get_info(h, &info), MLBM_OK);
    if (info.lattice != 19 || info.ncell != 13 * 9 * 11) ++failures;
    EXPECT(mlbm_get_info(h, NULL), MLBM_EINVAL);
    size_t fb = 0;
    EXPECT(mlbm_field_bytes(h, &fb), MLBM_OK);
    if (fb != (size_t)4 * 19 * 13 * 9 * 11 * 8) ++failures;

    EXPECT(mlbm_set_tau(h, 0.9), MLBM_OK);
    EXPECT(mlbm_set_tau(h, 0.4), MLBM_EDOMAIN);
    EXPECT(mlbm_set_eq_mode(h, MLBM_EQ_EIGEN), MLBM_OK);
    EXPECT(mlbm_set_positivity(h, 1), MLBM_EINVAL);
    EXPECT(mlbm_set_eq_mode(h, MLBM_EQ_ISOTHERMAL), MLBM_OK);
    EXPECT(mlbm_set_positivity(h, 1), MLBM_OK);
    EXPECT(mlbm_set_eq_mode(h, 9), MLBM_EINVAL);
    EXPECT(mlbm_set_eq_mode(h2, MLBM_EQ_EIGEN), MLBM_EINVAL);          /* eigen mode needs double */
    EXPECT(mlbm_set_positivity(h, 0), MLBM_OK);
    EXPECT(mlbm_set_eq_mode(h, MLBM_EQ_DIRECT), MLBM_OK);
    const double b[3] = {0.1, -0.2, 0.3}, zb[3] = {0.0, 0.0, 0.0};
    EXPECT(mlbm_set_magnetic_field(h, b), MLBM_OK);
    EXPECT(mlbm_set_positivity(h, 1), MLBM_EINVAL);
    EXPECT(mlbm_set_eq_mode(h, MLBM_EQ_ISOTHERMAL), MLBM_EINVAL);
    EXPECT(mlbm_set_magnetic_field(h, zb), MLBM_OK);
    EXPECT(mlbm_set_magnetic_field_map(h, NULL), MLBM_OK);
    EXPECT(mlbm_set_launch(h, 64, MLBM_ORDER_NATURAL, 2), MLBM_OK);
    EXPECT(mlbm_set_launch(h, 96, MLBM_ORDER_NATURAL, 2), MLBM_EINVAL);
    EXPECT(mlbm_set_launch(h, 64, 5, 2), MLBM_EINVAL);
    EXPECT(mlbm_set_launch(h, 64, MLBM_ORDER_AUTO, 40), MLBM_EINVAL);
    EXPECT(mlbm_set_launch(h, 0, MLBM_ORDER_AUTO, -1), MLBM_OK);
    double ref[4 * 19];
    for (int j = 0; j < 4 * 19; ++j) ref[j] = 0.01 * j;
    EXPECT(mlbm_set_f16_reference(h16, ref, 0.5), MLBM_OK);
    EXPECT(mlbm_set_f16_reference(h16, ref, 0.0), MLBM_EINVAL);
    EXPECT(mlbm_set_f16_reference(h, ref, 0.5), MLBM_EINVAL);          /* not an F16 handle */

    /* compute entry points: argument checks only (fake pointers are never dereferenced) */
    void* p1 = (void*)0x1000;
    void* p2 = (void*)0x2000;
    EXPECT(mlbm_step(h, NULL, p2, 3, NULL), MLBM_EINVAL);
    EXPECT(mlbm_step(h, p1, p1, 3, NULL), MLBM_EINVAL);
    EXPECT(mlbm_step(h, p1, p2, -1, NULL), MLBM_EINVAL);
    EXPECT(mlbm_step(h, p1, p2, 0, NULL), MLBM_OK);
    EXPECT(mlbm_stream(h, p1, p1, NULL), MLBM_EINVAL);
    EXPECT(mlbm_adjoint_step(h, p1, p2, p2, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_adjoint_step(h16, p1, p2, (void*)0x3000, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_adjoint_segment(h, p1, NULL, 0, p2, (void*)0x3000, NULL, NULL), MLBM_OK);
    EXPECT(mlbm_adjoint_segment(h, p1, NULL, 2, p2, (void*)0x3000, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_init_equilibrium(h, p1, NULL, p2, p2, NULL), MLBM_EINVAL);
    EXPECT(mlbm_init_chemical(h, p1, NULL, NULL, p2, p2, NULL), MLBM_EINVAL);
    EXPECT(mlbm_relaxation(h, p1, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_spin_loss(h16, p1, p2, NULL, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_step_states(h, p1, p1, (void*)0x100000, 2, 3, NULL), MLBM_EINVAL);
    EXPECT(mlbm_step_states(h, p1, p2, NULL, 2, 3, NULL), MLBM_EINVAL);
    EXPECT(mlbm_step_states(h, p1, p2, (void*)0x100000, 1, 3, NULL), MLBM_EINVAL);
    EXPECT(mlbm_step_states(h, p1, p2, (void*)0x100000, 2, -1, NULL), MLBM_EINVAL);
    EXPECT(mlbm_adjoint_sweep(h, p1, NULL, 0, p2, (void*)0x3000, NULL, NULL), MLBM_OK);
    EXPECT(mlbm_adjoint_sweep(h, p1, NULL, 2, p2, (void*)0x3000, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_adjoint_sweep(h16, p1, p2, 2, (void*)0x3000, (void*)0x4000, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_set_store_policy(h, 1), MLBM_OK);
    EXPECT(mlbm_set_store_policy(h, 3), MLBM_EINVAL);
    EXPECT(mlbm_set_store_policy(h, -1), MLBM_OK);
    EXPECT(mlbm_set_adjoint_launch(h, MLBM_ADJ_CHANNEL, 128, MLBM_ORDER_XCD_RANGE, 1, 0), MLBM_OK);
    EXPECT(mlbm_set_adjoint_launch(h, 3, 0, MLBM_ORDER_AUTO, -1, -1), MLBM_EINVAL);
    EXPECT(mlbm_set_adjoint_launch(h, MLBM_ADJ_AUTO, 32, MLBM_ORDER_AUTO, -1, -1), MLBM_EINVAL);
    EXPECT(mlbm_set_adjoint_launch(h, MLBM_ADJ_AUTO, 0, MLBM_ORDER_AUTO, 33, -1), MLBM_EINVAL);
    EXPECT(mlbm_set_adjoint_launch(h, MLBM_ADJ_AUTO, 0, MLBM_ORDER_AUTO, -1, 2), MLBM_EINVAL);
    EXPECT(mlbm_set_adjoint_launch(h, MLBM_ADJ_AUTO, 0, MLBM_ORDER_AUTO, -1, -1), MLBM_OK);
    EXPECT(mlbm_step_post(h, NULL, 0, p2, NULL, 0, 1, NULL), MLBM_EINVAL);                 /* null src */
    EXPECT(mlbm_step_post(h, p1, 2, p2, NULL, 0, 1, NULL), MLBM_EINVAL);                   /* src_post */
    EXPECT(mlbm_step_post(h, p1, 0, p2, NULL, 0, -1, NULL), MLBM_EINVAL);                  /* nsteps < 0 */
    EXPECT(mlbm_step_post(h, p1, 0, p2, NULL, 0, 0, NULL), MLBM_OK);                       /* nothing to do */
    EXPECT(mlbm_step_post(h, p1, 0, p2, NULL, 0, 2, NULL), MLBM_EINVAL);                   /* missing states */
    EXPECT(mlbm_step_post(h, p1, 0, NULL, (void*)0x100000, 1, 3, NULL), MLBM_EINVAL);      /* nstates < 2 */
    EXPECT(mlbm_step_post(h, p1, 0, p1, NULL, 0, 1, NULL), MLBM_EINVAL);                   /* dst = src */
    EXPECT(mlbm_step_post(h, (void*)0x100000, 0, p2, (void*)0x100000, 2, 3, NULL), MLBM_EINVAL); /* src in states */
    EXPECT(mlbm_adjoint_sweep_post(h, p1, NULL, 0, p2, (void*)0x3000, NULL, NULL), MLBM_OK);
    EXPECT(mlbm_adjoint_sweep_post(h, p1, NULL, 2, p2, (void*)0x3000, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_adjoint_sweep_post(h16, p1, p2, 2, (void*)0x3000, (void*)0x4000, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_moments_noalloc(NULL, p1, NULL, NULL, NULL, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_moments_noalloc(h, NULL, NULL, NULL, NULL, NULL, NULL), MLBM_EINVAL);
    EXPECT(mlbm_device_copy(NULL, p2, 64, NULL), MLBM_EINVAL);
    EXPECT(mlbm_device_copy(p1, p2, 24, NULL), MLBM_EINVAL);                /* not a multiple of 16 */
    EXPECT(mlbm_device_copy((void*)0x1008, p2, 64, NULL), MLBM_EINVAL);     /* misaligned */
    EXPECT(mlbm_device_copy(p1, (void*)0x1040, 128, NULL), MLBM_EINVAL);    /* overlapping */
    EXPECT(mlbm_device_copy(p1, p2, 0, NULL), MLBM_OK);                     /* nothing to copy */

    mlbm_destroy(h);
    mlbm_destroy(h2);
    mlbm_destroy(h16);
    mlbm_destroy(NULL);
    if (failures) fprintf(stderr, "%d unexpected status codes\n", failures);
    else printf("host checks passed\n");
    return failures ? 1 : 0;
}
