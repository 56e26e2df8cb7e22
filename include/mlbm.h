/*
 * mlbm.h -- C ABI of the matrix-valued quantum lattice Boltzmann library for
 * AMD Instinct MI355X (gfx950).
 *
 * The method is Mendl, "Matrix-valued Quantum Lattice Boltzmann Method"
 * (arXiv:1309.1656), Sec. 3.  Every population W_i(x) is a 2x2 complex
 * Hermitian spin-density matrix (Sec. 2, after Eq. BoltzmannEquation), held
 * here as four real Pauli coefficients
 *     W = (a0 I + a1 sigma_x + a2 sigma_y + a3 sigma_z) / 2,
 * so a0 = tr W and ak = tr(W sigma_k) (the Bloch components of Sec. 4).
 *
 * ---------------------------------------------------------------------------
 * Lattices and velocity order (Sec. 3, Fig. 1; Sec. 3.1).  e_i = xi * c_i.
 *   D2Q9  (Q = 9):  0:(0,0)  1:(1,0) 2:(-1,0) 3:(0,1) 4:(0,-1)
 *                   5:(1,1) 6:(-1,-1) 7:(1,-1) 8:(-1,1)
 *   D3Q19 (Q = 19): 0:(0,0,0)
 *                   1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1) 6:(0,0,-1)
 *                   7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0)
 *                   11:(1,0,1) 12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1)
 *                   15:(0,1,1) 16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1)
 *   Components are (x, y[, z]).  Weights: D2Q9 {1-5a, a, a/4}, D3Q19
 *   {1-12a, a, a/2} by number of nonzero components (Eqs. QuadSolution2D/3D at
 *   mu0 = 0, Eqs. QuadSolution2Dmu0 / QuadSolution3Dmu0).
 *
 * Field layout ("a field").  Row-blocked structure of arrays: cells are
 * grouped in x-rows, row = y + ny * z, and each row holds 4 * Q contiguous
 * segments of nx values, one per (Pauli component k, velocity i):
 *     element (k, i, x, y, z) at ((row * 4 + k) * Q + i) * nx + x,
 * i.e. a C-contiguous array [nz][ny][4][Q][nx] of the storage type (nz = 1
 * in 2D).  Lanes along x access consecutive addresses, and one row's update
 * writes one contiguous block.  Periodic boundaries in every direction
 * (Sec. 3).  Per-cell arrays (rho4, u, T, eps, r_target) are plain planes
 * [rows][N] with cell = x + nx * (y + ny * z).  Storage types:
 *   MLBM_STORE_F64     double; all arithmetic in double.
 *   MLBM_STORE_F32     float; collision arithmetic in float, moment sums in
 *                      double.  The conservation defect of each cell's
 *                      rounded outputs (mass per Pauli component, momentum,
 *                      energy) is summed in double and folded back into the
 *                      rest and axis populations, so the rounding of the float
 *                      constants does not make the global averages drift.
 *   MLBM_STORE_F16DEV  IEEE binary16 h = (a - R_ki) / s_i, the scaled
 *                      deviation from a lattice-weighted reference
 *                      equilibrium R_ki = w_i rho_bar_k P_i(u_bar, eps_bar) of
 *                      the global means of the initial state.  S is the power
 *                      of two at or above max |a - R| / w_i over the initial
 *                      field, and s_i = 2^round(log2(w_i S)) (|h| <= sqrt 2
 *                      initially; both scalings are exact).  R and S are fixed
 *                      by mlbm_init_equilibrium (or mlbm_init_chemical) and
 *                      kept in the handle.
 *                      Encoding rounds to nearest even; arithmetic in float,
 *                      moment sums in double.
 *
 * Time stepping (Sec. 3.3): Delta t = 1, Delta x = xi, omega = 1/tau.  One step
 * computes per cell the moments rho, u, eps (Eq. DiscrAvr), the polynomial
 * equilibrium W_eq_i = w_i rho P_i(u, eps) (Eq. WeqAlgo, Appendix
 * coefficients with eps_FD = eps), the BGK collision (Eq. CollisionStep) and
 * the periodic streaming W_i(x + c_i) <- W_coll_i(x) (Eq. TransportStep).
 *
 * Memory ownership.  Every field and every per-cell array passed to the
 * library is caller-owned DEVICE memory (for instance a torch tensor),
 * contiguous, aligned to at least 16 bytes, on the current HIP device.  The
 * handle owns only its constants, the F16DEV reference and scale, and a small
 * private device buffer for reductions and status flags (allocated on first
 * use).  Pointers documented as "host" are ordinary host memory.
 *
 * Streams.  Every call that takes `stream` (a hipStream_t; NULL means the
 * null stream) enqueues its work asynchronously on that stream and returns.
 * The exceptions synchronise `stream` and say so: mlbm_init_equilibrium and
 * mlbm_init_chemical (read back status flags), mlbm_relaxation (host output)
 * and mlbm_moments when a host output is requested.
 * A handle must not be used by two host threads at once; calls on one handle
 * on different streams must be ordered by the caller.
 *
 * Errors.  Every call returns MLBM_OK (0) or a negative status.  When argument
 * validation fails nothing is enqueued.  mlbm_last_error() returns a message
 * describing the last failure on the calling thread.
 */
#ifndef MLBM_H
#define MLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlbm_ctx* mlbm_handle;

enum { MLBM_D2Q9 = 9, MLBM_D3Q19 = 19 };
enum { MLBM_STORE_F64 = 0, MLBM_STORE_F32 = 1, MLBM_STORE_F16DEV = 2 };
enum { MLBM_EQ_DIRECT = 0, MLBM_EQ_EIGEN = 1, MLBM_EQ_ISOTHERMAL = 2 };
enum { MLBM_ORDER_AUTO = -1, MLBM_ORDER_NATURAL = 0, MLBM_ORDER_XCD_RANGE = 1, MLBM_ORDER_INTERLEAVE8 = 2 };
enum { MLBM_ADJ_AUTO = 0, MLBM_ADJ_CHANNEL = 1, MLBM_ADJ_CELL = 2 };
enum {
    MLBM_OK = 0,
    MLBM_EINVAL = -1,     /* bad argument: null pointer, bad enum, bad size   */
    MLBM_EDOMAIN = -2,    /* outside the method's domain (tau <= 1/2, ...)   */
    MLBM_EHIP = -3,       /* HIP runtime failure; message has hipGetErrorString */
    MLBM_ENOMEM = -4,     /* device allocation of the private buffer failed   */
    MLBM_ENONFINITE = -5, /* a NaN or infinity was found in a field           */
    MLBM_ENOCONV = -6     /* a Fermi-Dirac parameter inversion did not converge */
};

/* Read-only description of a handle (mlbm_get_info). */
typedef struct {
    int lattice;          /* MLBM_D2Q9 or MLBM_D3Q19 (= Q)                    */
    int d;                /* 2 or 3                                           */
    int storage;          /* MLBM_STORE_*                                      */
    int eq_mode;          /* MLBM_EQ_*                                         */
    int64_t nx, ny, nz;   /* grid; nz = 1 for D2Q9                             */
    int64_t ncell;        /* N = nx * ny * nz                                  */
    double tau, omega;    /* relaxation time and omega = Delta t / tau         */
    double beta0;         /* reference inverse temperature of the cubature    */
    double xi;            /* lattice constant = lattice speed, xi1 / sqrt(beta0) */
    double a;             /* cubature weight parameter at mu0 = 0              */
    double w[19];         /* weight of velocity i (first Q entries used)       */
    int c[19][3];         /* integer velocity c_i (x, y, z)                    */
    /* Appendix coefficients: alpha1 = a1_0 + a1_b b, alpha2 = a2_0 + a2_b b,
     * b = beta0 eps; alpha3..alpha5 constant.                                 */
    double a1_0, a1_b, a2_0, a2_b, a3, a4, a5;
    int launch_block_x;   /* step kernels: cells per workgroup along x (64, 128) */
    int launch_order;     /* step kernels: block order (MLBM_ORDER_*)          */
    double f16_scale;     /* S of MLBM_STORE_F16DEV (0 before initialisation) */
    double f16_ref[4][19];/* R_ki of MLBM_STORE_F16DEV                          */
    int launch_blocks_per_cu; /* step kernels: resident workgroups per CU (0: hardware limit) */
    int launch_temporal_stores; /* step kernels: 1 temporal field writes, 0 streaming */
    int adjoint_form;     /* adjoint kernels: MLBM_ADJ_CHANNEL or MLBM_ADJ_CELL in effect */
    int adjoint_block_x;  /* channel form: cells per workgroup along x (0 in the cell form) */
    int adjoint_order;    /* channel form: block order (MLBM_ORDER_*; -1 in the cell form) */
    int adjoint_blocks_per_cu;   /* channel form: resident workgroups per CU (0: hardware limit) */
    int adjoint_temporal_stores; /* channel form: 1 temporal writes of lam_n, 0 streaming */
} mlbm_info;

/*
 * mlbm_create -- set up a lattice of dims = {nx, ny, nz} cells (nz = 1 for
 * D2Q9), relaxation time tau (Eq. C_BGK, Eq. CollisionStep) and reference
 * inverse temperature beta0 of the cubature (Sec. 3.3, first paragraph;
 * mu0 = 0).  Computes xi, w_i and the Appendix coefficients in double on the
 * host.  Touches no device memory.
 *   lattice  MLBM_D2Q9 or MLBM_D3Q19.   storage  MLBM_STORE_*.
 *   Each dim >= 1, nx <= 2^29, ny and nz <= 65535, and N < 2^31.
 * Errors: MLBM_EINVAL (null out/dims, bad lattice/storage/dims),
 *         MLBM_EDOMAIN (tau <= 1/2 or not finite, beta0 <= 0 or not finite).
 *         tau > 1/2 keeps |1 - omega| < 1.
 * On success *out holds a new handle; release it with mlbm_destroy.
 */
int mlbm_create(mlbm_handle* out, int lattice, const int64_t dims[3],
                double tau, double beta0, int storage);

/* mlbm_destroy -- free the handle and its private device buffer (NULL is a no-op). */
void mlbm_destroy(mlbm_handle h);

/* mlbm_get_info -- copy the handle's parameters into *info (host). */
int mlbm_get_info(mlbm_handle h, mlbm_info* info);

/* mlbm_field_bytes -- bytes of one field: 4 * Q * N * sizeof(storage type). */
int mlbm_field_bytes(mlbm_handle h, size_t* bytes);

/* mlbm_set_tau -- change the relaxation time (same rules as mlbm_create). */
int mlbm_set_tau(mlbm_handle h, double tau);

/*
 * mlbm_set_eq_mode -- choose how the collision builds W_eq.
 *   MLBM_EQ_DIRECT (default): Eq. WeqAlgo, W_eq_i = w_i rho P_i(u, eps); no U,
 *     no Fermi-Dirac integral (Sec. 3.3, first item).
 *   MLBM_EQ_EIGEN: Eq. WeqDiscr taken literally: per cell the closed-form
 *     eigen-decomposition of rho gives U and the channel densities, a
 *     double-precision Newton inversion gives (beta, nu_up, nu_dn) with those
 *     densities and internal energy eps (Prop. 1), and
 *     W_eq_i = w_i U diag(n_up, n_dn) U* P_i(u, eps_FD) is rebuilt from them.
 *     Equal to the direct form up to the inversion tolerance; a checking mode,
 *     many times slower.  Only for MLBM_STORE_F64 (else MLBM_EINVAL).
 *   MLBM_EQ_ISOTHERMAL: the isothermal model the paper mentions and sets
 *     aside (Sec. 3.1, paragraph on beta0 and mu0): every cell's equilibrium
 *     has beta = beta0.  Per cell the eigenvalues n_up/dn = (tr rho +- |rho|)/2
 *     are inverted to nu at beta0 (Eq. nFDstdOmega, in double) and the
 *     Appendix coefficients take eps_FD(beta0; nu_up, nu_dn) of
 *     Eq. energyFDstdOmega instead of the moment eps.  Mass and momentum are
 *     conserved, energy is not.  Needs every cell's rho positive definite
 *     (otherwise the result is not finite, which mlbm_moments reports).
 * Errors: MLBM_EINVAL (bad mode; EIGEN without double storage or with the
 * positivity limit; a mode other than DIRECT while a magnetic field is set).
 */
int mlbm_set_eq_mode(mlbm_handle h, int mode);

/*
 * mlbm_set_positivity -- on = 1: positivity-limited relaxation, the
 * adjustment the paper describes and avoids (Sec. 3.3, paragraph after the
 * algorithm).  Per cell the collision uses the largest omega' in [0, omega]
 * such that for every population i the smaller eigenvalue of
 * (1 - omega') W_i + omega' W_eq_i is at least min(0, smaller eigenvalue of
 * W_i): positive semidefinite populations stay so, and one that is already
 * slightly negative (rounding) is not made worse.  The bound of each
 * population is the first downward zero of a quadratic in omega' (the
 * smaller eigenvalue is concave in omega'), the cell takes the minimum.
 * Mass, momentum and energy stay conserved (omega' is one number per cell).
 * on = 0 restores the plain BGK step.  Combines with MLBM_EQ_DIRECT and
 * MLBM_EQ_ISOTHERMAL; not with MLBM_EQ_EIGEN, a magnetic field or the
 * adjoint (MLBM_EINVAL).  The variant kernels use 64-cell blocks.
 */
int mlbm_set_positivity(mlbm_handle h, int on);

/*
 * mlbm_init_equilibrium -- write into field W the discrete Fermi-Dirac
 * equilibrium of per-cell macroscopic data (Eq. WeqDiscr; Eqs. WFermiDirac,
 * nFDstdOmega, energyFDstdOmega):
 *   rho4 [4][N] double (device): tr rho, r_x, r_y, r_z, where r is the Bloch
 *        vector r_k = tr(rho sigma_k), so rho = (tr rho I + r . sigma) / 2;
 *   u    [d][N] double (device): velocity in momentum units (the lattice speed
 *        is xi);
 *   T    [N]    double (device): temperature 1 / beta.
 * Per cell the channel densities n_up/dn = (tr rho +- |r|)/2 are inverted to
 * nu = beta mu by n = (2 pi / beta)^(d/2) F_{d/2-1}(nu) (closed form for d = 2,
 * Newton in double for d = 3), eps = (d/2) T sum F_{d/2}(nu) / sum F_{d/2-1}(nu),
 * and W_i = w_i rho P_i(u, eps).  For MLBM_STORE_F16DEV the routine first
 * reduces the global means and the maximal deviation to fix R and S.
 * Synchronises `stream` (reads back status flags).
 * Errors: MLBM_EINVAL (null pointers), MLBM_EDOMAIN (some cell has tr rho <= 0,
 * |r| >= tr rho, T <= 0, or a non-finite input), MLBM_ENOCONV (Newton failed),
 * MLBM_EHIP.  After a device-side EDOMAIN / ENOCONV the content of W is
 * unspecified.
 */
int mlbm_init_equilibrium(mlbm_handle h, void* W, const double* rho4,
                          const double* u, const double* T, void* stream);

/*
 * mlbm_init_chemical -- the same discrete Fermi-Dirac equilibrium, with each
 * cell named by its chemical potentials as in the Riemann problem of Sec. 4:
 *   nu   [2][N] double (device): nu_up = beta mu_up and nu_dn = beta mu_dn;
 *   axis [3][N] double (device) or NULL: the spin axis a of the up channel
 *        (any nonzero length, normalised per cell); NULL means +z;
 *   u, T as for mlbm_init_equilibrium.
 * Per cell n_up/dn = (2 pi / beta)^(d/2) F_{d/2-1}(nu_up/dn) (Eq. nFDstdOmega),
 * rho = U diag(n_up, n_dn) U* = ((n_up + n_dn) I + (n_up - n_dn) a . sigma)/2,
 * eps as above (Eq. energyFDstdOmega), W_i = w_i rho P_i(u, eps).
 * Synchronises `stream`.  Errors: MLBM_EINVAL (null W, nu, u or T),
 * MLBM_EDOMAIN (some cell has T <= 0, a zero or non-finite axis, nu > 4000 or
 * a non-finite input), MLBM_EHIP.  F16DEV reference and scale as above.
 */
int mlbm_init_chemical(mlbm_handle h, void* W, const double* nu, const double* axis, const double* u,
                       const double* T, void* stream);

/*
 * mlbm_step -- advance W by nsteps >= 0 time steps (Sec. 3.3).  W holds the
 * pre-collision state W(t) on entry and W(t + nsteps) on exit.  `scratch` is a
 * second field of the same size, distinct from W, clobbered.  Implementation,
 * ping-ponging between W and scratch so that no copy is made: for nsteps >= 2,
 * one collide-only pass, nsteps - 2 fused pull-stream + collide passes and one
 * fused pass that writes each collided value where the step's final streaming
 * sends it (x + c_i), into W: nsteps passes in all.  For nsteps = 1, and in the
 * eigen-channel mode, one collide-only pass, nsteps - 1 fused passes and one
 * stream-only pass.  The state is the same bit for bit either way.
 * The collision is the one configured on the handle (equilibrium mode,
 * positivity limit, magnetic field).  Only kernel launches are enqueued (no
 * allocation, memset or synchronisation), so the call can be captured in a
 * HIP graph and replayed.
 * Errors: MLBM_EINVAL (null or equal pointers, nsteps < 0), MLBM_EHIP.
 */
int mlbm_step(mlbm_handle h, void* W, void* scratch, int nsteps, void* stream);

/*
 * mlbm_step_states -- the same nsteps time steps (Sec. 3.3) out of place,
 * keeping the intermediate states.  src holds the pre-collision state W(t)
 * and is only read; dst receives W(t + nsteps).  `states` is caller-owned
 * device memory for nstates fields laid out one after the other: the
 * post-collision state of step j (j = 0 .. nsteps - 1) is written to field
 * j mod nstates, so nstates >= nsteps keeps all of them (the layout
 * mlbm_adjoint_sweep reads) and nstates = 2 is a plain ping-pong.  Passes:
 * one collide-only, nsteps - 1 fused, one stream-only (every post-collision
 * state is kept, so the last one is streamed by a pass of its own); the same
 * values as mlbm_step bit for bit; no copy, except that nsteps = 0 copies src
 * to dst.  Only kernel launches (or
 * that one copy) are enqueued.
 * Errors: MLBM_EINVAL (null pointers, nsteps < 0, nstates < 1, or < 2 with
 * more than one step, src = dst, src or dst inside the states), MLBM_EHIP.
 */
int mlbm_step_states(mlbm_handle h, const void* src, void* dst, void* states, int nstates, int nsteps,
                     void* stream);

/*
 * mlbm_collide -- dst = C(src), the BGK collision of Eq. CollisionStep cell
 * by cell (as configured on the handle), no streaming.  dst may equal src
 * (in place).
 */
int mlbm_collide(mlbm_handle h, const void* src, void* dst, void* stream);

/*
 * mlbm_stream -- dst_i(x) = src_i(x - c_i), the periodic transport of
 * Eq. TransportStep alone.  A pure permutation of the stored values (bit
 * exact in every storage type).  dst must not overlap src.
 */
int mlbm_stream(mlbm_handle h, const void* src, void* dst, void* stream);

/*
 * mlbm_moments -- per-cell and global moments of a field W (Eq. DiscrAvr;
 * Eqs. GlobalDensity, GlobalVelocity, GlobalTotalEnergy).  Each output may be
 * NULL.
 *   rho4 [4][N] double (device): Pauli coefficients of rho = sum_i W_i;
 *   u    [d][N] double (device): velocity, tr(rho) u = sum_i e_i tr W_i;
 *   eps  [N]    double (device): internal energy,
 *        tr(rho) eps = sum_i |e_i - u|^2/2 tr W_i;
 *   global8 [8] double (host): cell averages of the 4 Pauli coefficients of
 *        rho, of tr(rho) u (3 entries, third 0 in 2D) and of
 *        tr(rho)(eps + |u|^2/2) = sum_i |e_i|^2/2 tr W_i;
 *   n_neg_eig [1] int64 (host): number of populations W_i(x) with a negative
 *        eigenvalue (a0 - |a| < 0; Sec. 3.2, last paragraph; Sec. 3.3).
 * Global sums are reduced in a fixed order (bitwise reproducible).  When a host
 * output is requested the call synchronises `stream`, and returns
 * MLBM_ENONFINITE (outputs still written) if any value of W is NaN or infinite.
 */
int mlbm_moments(mlbm_handle h, const void* W, double* rho4, double* u,
                 double* eps, double* global8, int64_t* n_neg_eig, void* stream);

/*
 * mlbm_moments_noalloc -- mlbm_moments for callers that cannot allocate
 * device memory or synchronise (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same kernels and fixed-order
 * reduction, with no host output, no allocation and no synchronisation.
 *   rho4, u, eps as for mlbm_moments (device, each may be NULL);
 *   sums [10] double (device) or NULL: the SUMS over cells (not averages) of
 *        the 4 Pauli coefficients of rho, of tr(rho) u (3 entries, third 0 in
 *        2D) and of tr(rho)(eps + |u|^2/2); then the number of populations
 *        with a negative eigenvalue and the number of non-finite values, as
 *        doubles.  Divided by N, entries 0..7 are mlbm_moments' global8.
 * The reduction buffer is a fixed-size array in device memory (1024 x 10
 * doubles, 80 KiB, whatever the lattice size) that each GPU holds from the
 * first call until the process ends; the first call on a device also looks
 * up its address.  Every call on one GPU shares that buffer, so calls that
 * overlap in time on one GPU (other streams, other handles, other host
 * threads) race: order them.  Non-finite values are counted, not reported as
 * an error.  Errors: MLBM_EINVAL (null handle or W), MLBM_EHIP.
 */
int mlbm_moments_noalloc(mlbm_handle h, const void* W, double* rho4, double* u,
                         double* eps, double* sums, void* stream);

/*
 * mlbm_relaxation -- how far field W is from the uniform state it relaxes to
 * (Sec. 4, convergence to equilibrium), and the split of the global energy
 * (Sec. 4, interference: the total is conserved, the internal part is not).
 * The uniform state has the global averages rho_bar, u_bar, eps_tot_bar of
 * Eqs. GlobalDensity, GlobalVelocity, GlobalTotalEnergy.  out[8] (host):
 *   out[0] max over cells of ||rho(x) - rho_bar|| (spectral norm of the 2x2
 *          Hermitian difference, (|d0| + |d|)/2 in Pauli coefficients d),
 *   out[1] max |u(x) - u_bar|,   out[2] max |eps_tot(x) - eps_tot_bar|,
 *          with eps_tot(x) = eps(x) + |u(x)|^2 / 2,
 *   out[3] mean over cells of tr rho(x) eps(x)       (internal energy),
 *   out[4] mean over cells of tr rho(x) |u(x)|^2 / 2 (kinetic energy),
 *   out[5..7] root mean square over cells of the distances of out[0..2].
 * Two reduction passes in fixed order (bitwise reproducible); synchronises
 * `stream`.  Errors: MLBM_EINVAL (null W or out), MLBM_ENONFINITE, MLBM_EHIP.
 */
int mlbm_relaxation(mlbm_handle h, const void* W, double out[8], void* stream);

/*
 * mlbm_spin_loss -- L = (1/N) sum_x |r(x) - r_target(x)|^2 with r the Bloch
 * vector of rho(x) = sum_i W_i(x), and its gradient with respect to W:
 *   r_target [3][N] double (device);
 *   loss     device double, overwritten with L (may be NULL);
 *   lam      device field of W's storage type (may be NULL): component k of
 *            every population set to dL/da_k = (2/N)(r_k - r_target_k) for
 *            k = 1..3 and to 0 for k = 0.
 * MLBM_STORE_F16DEV is rejected (MLBM_EINVAL).
 */
int mlbm_spin_loss(mlbm_handle h, const void* W, const double* r_target,
                   double* loss, void* lam, void* stream);

/*
 * mlbm_adjoint_step -- reverse-mode derivative of one step W_{n+1} =
 * S(C(W_n)) (Eqs. CollisionStep, TransportStep):
 *   W_n       field, the pre-collision state of step n (device);
 *   lam_next  field, dL/da of W_{n+1} (device);
 *   lam_n     field, written with dL/da of W_n (device; must not overlap the
 *             inputs);
 *   dL_domega device double: the step's partial derivative with respect to
 *             omega = 1/tau is ADDED to it (dL/dtau = -dL/domega / tau^2).
 * Derivative, with g_i(x) = lam_next_i(x + c_i) and G_i = w_i sum_k g_ik rho_k:
 *   lam_n_jk = (1-omega) g_jk + omega sum_i w_i P_i g_ik
 *              + [k = 0] omega (G_u.(e_j - u) + G_eps(|e_j - u|^2/2 - eps)) / tr rho,
 *   G_u = sum_i G_i dP_i/du,  G_eps = sum_i G_i dP_i/deps,
 *   dL/domega += sum_{x,i,k} g_ik (W_eq_ik - a_ik).
 * With a magnetic field the Bloch part of g is first turned back by the
 * transpose of the cell's rotation.  Storage MLBM_STORE_F64 or MLBM_STORE_F32
 * (float fields, double sums); MLBM_STORE_F16DEV, an equilibrium mode other
 * than MLBM_EQ_DIRECT and the positivity limit are rejected (MLBM_EINVAL).
 */
int mlbm_adjoint_step(mlbm_handle h, const void* W_n, const void* lam_next,
                      void* lam_n, double* dL_domega, void* stream);

/*
 * mlbm_set_magnetic_field -- uniform external magnetic field (Sec. 5,
 * Eq. sigmaB_comm): the commutator -i [mu sigma.B, W] joins the collision.
 * mu_b[3] (host) is the product mu B of magnetic moment and field; NULL or
 * zero switches the field off.  Reading: over each time step the commutator
 * is integrated exactly, W_i -> U W_i U* with U = exp(-i Delta t sigma.(mu B)),
 * i.e. every Bloch vector turns by 2 Delta t |mu B| about B; it commutes with
 * the BGK collision of a cell, so the order of the two does not matter.
 * Traces (density, momentum, energy) are untouched; tr(rho sigma) precesses.
 * Needs MLBM_EQ_DIRECT without the positivity limit (MLBM_EINVAL).  The
 * adjoint entry points follow the field: the Bloch part of the adjoint is
 * turned back by the transpose of each cell's rotation before the
 * collision's adjoint.
 */
int mlbm_set_magnetic_field(mlbm_handle h, const double mu_b[3]);

/*
 * mlbm_set_magnetic_field_map -- spatially varying field: mu_b is caller-owned
 * device memory [3][N] (double, plain cell order) holding mu B per cell,
 * read by every later step (update it between steps for a time-dependent
 * field); NULL switches the field off.  Same reading and restrictions as
 * mlbm_set_magnetic_field.
 */
int mlbm_set_magnetic_field_map(mlbm_handle h, const double* mu_b);

/*
 * mlbm_set_launch -- launch shape of the step kernels (performance only; the
 * results are identical).  Each workgroup covers block_x consecutive cells
 * of one x-row with four waves per 64 cells, one per Pauli component
 * (block_x = 64 or 128; 0 = automatic).  order chooses how workgroups map to
 * the 8 XCDs of the chip, each with its own L2 (MLBM_ORDER_NATURAL: x-chunk
 * fastest; MLBM_ORDER_XCD_RANGE: a contiguous range of rows per XCD;
 * MLBM_ORDER_INTERLEAVE8: 8 rows across the XCDs, the chunks of a row on one
 * XCD; MLBM_ORDER_AUTO: chosen from the grid size and storage type).
 * blocks_per_cu caps the workgroups resident on one CU (1..32) by reserving
 * unused LDS: fewer waves in flight means fewer concurrent DRAM streams,
 * which raises the bandwidth the pass reaches; 0 = no cap (hardware limit),
 * -1 = automatic.  The automatic shape depends on the kernel in use too: the
 * magnetic-field and variant kernels (the variants always in 64-cell blocks)
 * take their own measured order and cap, and the last pass of mlbm_step
 * (which writes pushed) takes 128-cell blocks in natural order when a row has
 * 65 to 128 cells, so that one workgroup writes a whole row (1 workgroup per
 * CU for D3Q19 FP64).  mlbm_get_info reports the shape of the other passes
 * in effect for the handle's current collision.
 * Errors: MLBM_EINVAL.
 */
int mlbm_set_launch(mlbm_handle h, int block_x, int order, int blocks_per_cu);

/*
 * mlbm_set_adjoint_launch -- launch shape of the adjoint kernels
 * (mlbm_adjoint_step, mlbm_adjoint_segment, mlbm_adjoint_sweep; performance
 * only, the values computed are the same up to the summation order of
 * dL/domega).  form: MLBM_ADJ_CHANNEL runs one wave per Pauli component on
 * block_x consecutive cells of one x-row, like the step kernels (block_x,
 * order, blocks_per_cu and stores as for mlbm_set_launch and
 * mlbm_set_store_policy); MLBM_ADJ_CELL runs one thread per cell with all
 * four components (the other arguments are then ignored); MLBM_ADJ_AUTO
 * chooses.  A magnetic field always uses the cell form.  mlbm_get_info
 * reports the shape in effect.  Errors: MLBM_EINVAL.
 */
int mlbm_set_adjoint_launch(mlbm_handle h, int form, int block_x, int order, int blocks_per_cu, int stores);

/*
 * mlbm_set_store_policy -- how the step passes write a field: -1 automatic
 * (the default: temporal when one field holds at most 192 MiB, streaming
 * above; an empirical cut-off from measured pass times, below which part of
 * what the next pass reads is found in the 256 MB last-level cache), 0
 * streaming (non-temporal) stores, 1 temporal stores.
 * The stored values are the same either way; the magnetic-field and variant
 * kernels always stream.  mlbm_get_info reports the policy in effect.
 * Errors: MLBM_EINVAL (policy outside -1..1).
 */
int mlbm_set_store_policy(mlbm_handle h, int policy);

/*
 * mlbm_adjoint_segment -- the adjoint of nsteps >= 0 consecutive steps in one
 * call, for checkpointed reverse mode.  W is the segment's first
 * pre-collision state (its checkpoint; read only).  The nsteps - 1
 * intermediate states are recomputed into `states`, caller-owned device
 * memory for nsteps - 1 fields laid out one after the other (may be NULL if
 * nsteps <= 1), in post-collision form (one fused pass each).  Then the
 * adjoint steps run from the last to the first, gathering each pre-collision
 * state from the previous post-collision one:
 *   lam      on entry dL/da of the state after the segment, on exit dL/da of W;
 *   lam_tmp  workspace field (clobbered);
 *   dL_domega device double, accumulated (+=) as in mlbm_adjoint_step.
 * Same derivative and restrictions as mlbm_adjoint_step; lam, lam_tmp and W
 * must be distinct.
 */
int mlbm_adjoint_segment(mlbm_handle h, const void* W, void* states, int nsteps, void* lam,
                         void* lam_tmp, double* dL_domega, void* stream);

/*
 * mlbm_adjoint_sweep -- the reverse half of mlbm_adjoint_segment: the same
 * nsteps adjoint steps, from the last to the first, with the intermediate
 * states already in `states` (fields 0 .. nsteps - 2: the post-collision
 * states of steps 0 .. nsteps - 2 after W, as mlbm_step_states writes them
 * with nstates >= nsteps - 1; read only).  For the segment whose states the
 * forward pass kept, so that it needs no recomputation.  Arguments, result
 * and restrictions otherwise as mlbm_adjoint_segment.
 */
int mlbm_adjoint_sweep(mlbm_handle h, const void* W, const void* states, int nsteps, void* lam,
                       void* lam_tmp, double* dL_domega, void* stream);

/*
 * mlbm_step_post -- nsteps time steps (Sec. 3.3) that keep only post-collision
 * states, for checkpointing in post-collision form.  src is the state to
 * advance from: the pre-collision state W(t) when src_post = 0, or the
 * post-collision state S(t - 1) of the previous step when src_post = 1 (then
 * W(t) is its streaming, Eq. TransportStep).  The post-collision state S(t + j)
 * of step j (j = 0 .. nsteps - 1) is written to field j mod nstates of
 * `states` (caller-owned device memory, fields one after the other), except
 * the last one, which goes to dst when dst is not NULL.  No streaming pass
 * follows: the pre-collision state W(t + nsteps) is mlbm_stream of the last
 * one.  Passes: one collide-only (src_post = 0) or fused (src_post = 1) pass,
 * then nsteps - 1 fused passes.  Only kernel launches are enqueued.  The
 * collision is the handle's (field, variants), except the eigen-channel mode.
 * Errors: MLBM_EINVAL (null src, src_post not 0 or 1, nsteps < 0, missing
 * states, nstates < 2 with more than one state kept, src or dst overlapping
 * the states written or each other, eigen-channel mode), MLBM_EHIP.
 */
int mlbm_step_post(mlbm_handle h, const void* src, int src_post, void* dst, void* states, int nstates,
                   int nsteps, void* stream);

/*
 * mlbm_adjoint_sweep_post -- mlbm_adjoint_sweep for a segment whose first
 * state is given in post-collision form: S_prev is the post-collision state of
 * the step before the segment (read only), so step 0 of the segment gathers
 * its pre-collision state from S_prev by a pull, as steps 1 .. nsteps - 1
 * gather theirs from states fields 0 .. nsteps - 2 (the post-collision states
 * that mlbm_step_post keeps).  Arguments, result and restrictions otherwise
 * as mlbm_adjoint_sweep.
 */
int mlbm_adjoint_sweep_post(mlbm_handle h, const void* S_prev, const void* states, int nsteps, void* lam,
                            void* lam_tmp, double* dL_domega, void* stream);

/*
 * mlbm_set_f16_reference -- restore the MLBM_STORE_F16DEV reference R (4*Q
 * doubles, [k][i], host) and scale S > 0 saved from mlbm_get_info, so that a
 * saved F16DEV field can be resumed on a new handle.
 */
int mlbm_set_f16_reference(mlbm_handle h, const double* ref, double scale);

/*
 * mlbm_device_copy -- diagnostic, not part of the method: a plain copy of
 * `bytes` bytes from src to dst (device memory, 16-byte aligned, not
 * overlapping; bytes a multiple of 16, at most 2^35), one 16-byte vector per
 * thread with streaming loads and stores, enqueued on `stream`.  Its rate is
 * the achievable-bandwidth reference next to the step's fraction of the HBM
 * peak.  MLBM_EINVAL on a violated requirement (nothing enqueued).
 */
int mlbm_device_copy(const void* src, void* dst, size_t bytes, void* stream);

/* mlbm_last_error -- message of the last failed call on this thread ("" if none). */
const char* mlbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLBM_H */
