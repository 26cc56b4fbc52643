/* mclbm.h - C ABI of the MI355X Monte Carlo KBC lattice Boltzmann library.
 *
 * The library evolves an ensemble of M independent samples of the randomized
 * Taylor-Green vortex (RTGV) with a D3Q27 or D3Q19 lattice Boltzmann scheme
 * whose collision is the entropic multi-relaxation (KBC) operator: the
 * non-equilibrium part of the populations is split into a shear part and a
 * higher-order part, the shear part relaxes with omega (fixed by the
 * viscosity), the higher-order part with omega*gamma/2, and gamma is chosen
 * per node and time step by the closed-form entropic condition. The
 * ensemble is the empirical measure of the paper's Monte Carlo method.
 *
 * Paper passages (arXiv 2608.23786):
 *   equilibrium, moments ........ eq. (equilibrium) and the density/momentum
 *                                  definitions that follow it
 *   collide-and-stream .......... eq. (lbIteration)
 *   KBC collision ............... eqs. (kbcCollision), (entropyControl),
 *                                 Table 1 (relaxation groups and omega)
 *   random initial data ......... eqs. (alpha_perturbation), (tgv_init_velo),
 *                                 (initialRTGV), (initialPopulations)
 *   Monte Carlo ensemble ........ eq. (statSolDisc) and the push-forward
 *                                 construction of section 4.1
 *   kinetic energy .............. eq. (dftCoeff) normalisation (energy per
 *                                 unit volume of u)
 *
 * Conventions shared by every call
 *   - Velocities: D3Q27 numbers its 27 velocities c in {-1,0,1}^3 by
 *     i = 9*(cx+1) + 3*(cy+1) + (cz+1); D3Q19 (the paper's lattice, section
 *     on the deterministic scheme) keeps the same order without the eight
 *     corner velocities (|cx| = |cy| = |cz| = 1). With q velocities the
 *     opposite of population k is q - 1 - k. Weights: D3Q27 8/27, 2/27,
 *     1/54, 1/216; D3Q19 1/3, 1/18, 1/36 (rest, axis, diagonal, corner).
 *   - Nodes: x_n = 2*pi*n/N, n = 0..N-1 per axis (periodic box [0, 2pi)^3).
 *     Fields are C-ordered [z][y][x] (x fastest); cell = (z*N + y)*N + x.
 *   - Random parameters: Y[m][24] in [-1, 1]; Y[m][p] multiplies the product
 *     a_i(2x) a_j(2y) a_k(2z) in velocity component alpha, with
 *     p = 8*alpha + 4*i + 2*j + k, a_0 = sin, a_1 = cos. The physical
 *     coefficients are X = amp * u0 * Y.
 *   - Units: lattice units. Re = u0 * L / nu with L = N / (2 pi) lattice
 *     units, so nu = u0 * N / (2 pi Re) and omega = 1 / (3 nu + 1/2).
 *   - Time: one tick advances every sample whose stride divides the tick
 *     index by one lattice Boltzmann step. "State at step n" is the
 *     post-stream population field after n steps; step 0 is the initial
 *     equilibrium.
 *
 * Memory and streams
 *   The caller owns all device memory (the workspace, outputs, checkpoint and
 *   backward buffers) and the HIP stream; the library borrows them. A context
 *   holds host-side metadata only; mclbm_destroy frees no device memory.
 *   All device work is enqueued on the context's stream; device outputs are
 *   valid once that stream has been synchronised. Calls that take host
 *   pointers for output synchronise the stream themselves.
 *   One context per stream; contexts are not thread-safe.
 *
 * Errors
 *   Every call returns an mclbm_status. Arguments are validated before any
 *   work is enqueued (MCLBM_ERR_ARG). HIP runtime failures give
 *   MCLBM_ERR_HIP. Calls out of order (e.g. step before init) give
 *   MCLBM_ERR_STATE. A non-finite density or velocity, or a non-positive
 *   equilibrium population, met by a collision sets a sticky per-sample flag
 *   that the next mclbm_reduce / mclbm_moments / mclbm_check reports as
 *   MCLBM_ERR_UNSTABLE. mclbm_last_error() returns a message for the last
 *   failing call of the calling thread.
 */
#ifndef MCLBM_H
#define MCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mclbm_ctx mclbm_ctx;

typedef enum {
  MCLBM_OK = 0,
  MCLBM_ERR_ARG = 1,
  MCLBM_ERR_OOM = 2,         /* a caller-provided buffer is too small */
  MCLBM_ERR_HIP = 3,
  MCLBM_ERR_STATE = 4,
  MCLBM_ERR_UNSTABLE = 5,
  MCLBM_ERR_UNSUPPORTED = 6
} mclbm_status;

typedef enum {
  MCLBM_FP64 = 0,            /* populations stored and computed in double */
  MCLBM_FP32_SHIFTED = 1     /* g = f - w stored and computed in float */
} mclbm_precision;

typedef enum {
  MCLBM_GAMMA_CLOSED_FORM = 0, /* eq. (entropyControl): first-order closed form (default) */
  MCLBM_GAMMA_EXACT = 1        /* eq. (kbc_entropy): minimiser of the discrete H-function */
} mclbm_stabiliser;

typedef enum {
  MCLBM_D3Q27 = 27,          /* 27 velocities; hom group: T and 17 moments of order 3-6 */
  MCLBM_D3Q19 = 19           /* 19 velocities; hom group: T, Q (order 3), A (order 4) of Table 1 */
} mclbm_lattice;

/* One sample of the ensemble. */
typedef struct {
  int32_t n;        /* lattice points per axis: a power of two, 8 <= n <= 1024 */
  double u0;        /* Taylor-Green amplitude in lattice units, 0 < u0 <= 0.2 */
  double re;        /* Reynolds number u0 * (n / 2pi) / nu, > 0 */
  double amp;       /* perturbation amplitude relative to u0, >= 0 */
  int32_t project;  /* 1: Leray-project the perturbation; 0: use it as drawn */
  int32_t stride;   /* the sample steps on every stride-th tick, a power of two >= 1 */
} mclbm_sample_desc;

/* Shear relaxation frequency of a sample (Table 1):
 * omega = 2 c_s^2 / (2 nu + c_s^2) = 1 / (3 nu + 1/2), nu = u0 * n / (2 pi re).
 * Returns 0 for invalid arguments. */
double mclbm_omega(int32_t n, double u0, double re);

/* Bytes of device workspace mclbm_create needs for this ensemble (0 if the
 * descriptors, the precision or the lattice are invalid). Population storage
 * is one in-place buffer of q * n^3 values per sample (q = lattice), plus
 * small tables. */
size_t mclbm_workspace_bytes(int32_t m, const mclbm_sample_desc* desc, int32_t precision, int32_t lattice);

/* Create a context for m samples (1 <= m <= 65536) on one lattice
 * (MCLBM_D3Q27 or MCLBM_D3Q19). `workspace` is device memory of at least
 * mclbm_workspace_bytes() bytes, 256-byte aligned; `hip_stream` is a
 * hipStream_t (NULL for the null stream). The descriptors are copied. */
mclbm_status mclbm_create(mclbm_ctx** out, int32_t m, const mclbm_sample_desc* desc, int32_t precision,
                          int32_t lattice, void* workspace, size_t workspace_bytes, void* hip_stream);

mclbm_status mclbm_destroy(mclbm_ctx* ctx);

/* Draw or take the random parameters and set every sample to step 0:
 * u0(x) = u0 [TGV(x) + amp * P s(Y)(x)], f = f^eq(1, u0(x)).
 * y_host: host array Y[m][24], or NULL to draw Y with SplitMix64 from `seed`
 * (state = seed; per draw: state += 0x9E3779B97F4A7C15, then the
 * 30/27/31-bit xor-shift-multiply finaliser; Y = 2*(draw >> 11)*2^-53 - 1,
 * sample by sample, parameter by parameter). Resets the tick counter. */
mclbm_status mclbm_init(mclbm_ctx* ctx, uint64_t seed, const double* y_host);

/* Copy the random parameters in use to the host: Y[m][24]. */
mclbm_status mclbm_get_y(const mclbm_ctx* ctx, double* y_host);

/* Set the physical viscosity eps of every sample (host array of m values,
 * eps = 1/Re with unit reference length and velocity); nu = u0 * n * eps / (2 pi). */
mclbm_status mclbm_set_viscosity(mclbm_ctx* ctx, const double* eps_host);

/* Advance `ticks` ticks. If record_every > 0, the reductions of
 * mclbm_reduce are taken of the state at the start of every tick t of this
 * call with t % record_every == 0 (t counted from the start of the call),
 * fused into that tick's collide-and-stream, and written as consecutive
 * records of m*8 doubles to records_dev (device); max_records bounds how
 * many fit. record_every must then be a multiple of every sample's stride
 * and of the tick counter's phase. */
mclbm_status mclbm_step(mclbm_ctx* ctx, int64_t ticks, int32_t record_every, double* records_dev,
                        int64_t max_records);

/* Density and velocity of one sample at its current step, in double:
 * rho_dev[n^3], u_dev[3][n^3] (device, may be NULL to skip). */
mclbm_status mclbm_moments(mclbm_ctx* ctx, int32_t sample, double* rho_dev, double* u_dev);

/* Per-sample reductions of the current state into red_dev[m][8] (device):
 * total mass sum(rho), total momentum sum(rho u) (3), kinetic energy
 * mean(|u|^2 / 2), and min / max / mean of the stabiliser gamma that the
 * next collision computes from this state. Accumulated in double. */
mclbm_status mclbm_reduce(mclbm_ctx* ctx, double* red_dev);

/* Report the sticky instability flags: *first_bad = lowest unstable sample
 * or -1. Returns MCLBM_ERR_UNSTABLE if any. */
mclbm_status mclbm_check(mclbm_ctx* ctx, int32_t* first_bad);

/* Populations f (not shifted) of one sample at its current step, in double,
 * layout [q][n^3] (device, q = the lattice's velocities). get copies out; set
 * replaces the state (the sample's step count is kept). */
mclbm_status mclbm_get_state(mclbm_ctx* ctx, int32_t sample, double* f_dev);
mclbm_status mclbm_set_state(mclbm_ctx* ctx, int32_t sample, const double* f_dev);

/* Populations f (not shifted, double) of `count` cells of one sample at its
 * current step: cells_dev[count] (device, int64 cell indices, each checked
 * against n^3 before anything is enqueued), f_dev[count][q] (device). */
mclbm_status mclbm_get_cells(mclbm_ctx* ctx, int32_t sample, const int64_t* cells_dev, int32_t count, double* f_dev);

/* Write NaN into population i (0 <= i < q) of cell `cell` of one sample
 * (failure-path tests). */
mclbm_status mclbm_poison(mclbm_ctx* ctx, int32_t sample, int64_t cell, int32_t i);

/* Checkpoint: a device copy of the whole ensemble state and its step
 * counters. mclbm_checkpoint_bytes gives the size; restore puts the context
 * back to exactly that state. */
size_t mclbm_checkpoint_bytes(const mclbm_ctx* ctx);
mclbm_status mclbm_checkpoint(mclbm_ctx* ctx, void* dst_dev, size_t bytes);
mclbm_status mclbm_restore(mclbm_ctx* ctx, const void* src_dev, size_t bytes);

/* Gradient of J = (1/m) sum_m KE_m(T) with respect to Y (discrete adjoint).
 * Requires every stride to be 1 and the context to be at tick 0 (just
 * initialised).
 *   mclbm_forward_ckpt runs `ticks` steps from step 0 and stores a copy of
 *     the state every `ckpt_every` steps in ckpt_dev;
 *   mclbm_backward then computes dJdY_dev[m][24] (device, double) and
 *     ke_dev[m] = KE_m(T) (device, may be NULL), recomputing each segment
 *     of ckpt_every steps from its checkpoint into work_dev.
 * Sizes come from mclbm_ckpt_bytes / mclbm_backward_work_bytes. The state
 * after backward is the forward state at T. mclbm_backward returns
 * MCLBM_ERR_STATE (nothing enqueued) when any call changed the state or its
 * dynamics after the last mclbm_forward_ckpt (init, step, restore,
 * set_state, set_viscosity, set_stabiliser, poison, autotune), or when
 * ckpt_dev holds checkpoints of another forward run (each forward writes a
 * token into the first 256 bytes of its checkpoint buffer). Both stabilisers: with the exact
 * one (mclbm_set_stabiliser) each reverse step recomputes the forward t and
 * differentiates it through its stationarity condition (implicit function
 * theorem), FP64 states only: near equilibrium the exact minimiser moves f*
 * by an amount that does not vanish with dh (the third-order part of
 * ln(f^eq / w) along dh), so its derivative grows like 1/|dh|, and FP32
 * rounding of dh there makes it meaningless (MCLBM_ERR_UNSUPPORTED). */
size_t mclbm_ckpt_bytes(const mclbm_ctx* ctx, int64_t ticks, int32_t ckpt_every);
size_t mclbm_backward_work_bytes(const mclbm_ctx* ctx, int32_t ckpt_every);
mclbm_status mclbm_forward_ckpt(mclbm_ctx* ctx, int64_t ticks, int32_t ckpt_every, void* ckpt_dev,
                                size_t ckpt_bytes);
mclbm_status mclbm_backward(mclbm_ctx* ctx, int64_t ticks, int32_t ckpt_every, const void* ckpt_dev,
                            size_t ckpt_bytes, void* work_dev, size_t work_bytes, double* dJdY_dev,
                            double* ke_dev);

/* Vector-Jacobian product of one step (collide, then stream: eq.
 * (lbIteration) with the collision of eqs. (kbcCollision),
 * (entropyControl), or eq. (kbc_entropy) for the exact stabiliser) at the
 * current state f_n of every sample: out = (d f_{n+1} / d f_n)^T lam, the
 * reverse step mclbm_backward applies (the state is not advanced). lam_dev,
 * out_dev: device, double, the samples one after another, each [q][n^3] in
 * the population order of mclbm_get_state (derivatives with respect to the
 * unshifted populations f); in FP32 ensembles lam is rounded to float and
 * the product is computed in float. work_dev: mclbm_step_vjp_work_bytes
 * bytes of device scratch (three state copies), owned by the caller. The
 * same restrictions as mclbm_backward: every stride 1 (else
 * MCLBM_ERR_UNSUPPORTED), the exact stabiliser in FP64 only. */
size_t mclbm_step_vjp_work_bytes(const mclbm_ctx* ctx);
mclbm_status mclbm_step_vjp(mclbm_ctx* ctx, const double* lam_dev, double* out_dev, void* work_dev,
                            size_t work_bytes);

/* Observables of one sample's current velocity field, in double:
 *   s2_dev[n/2]: second-order structure function S2(r), r = 1..n/2, by the
 *     discrete Wiener-Khinchin route of Lemma (structureFunctionSpectral) /
 *     Algorithm 1: R_h = N^-3 F^-1(sum_a |F u_a|^2)_h (F unnormalised, F^-1
 *     with 1/N^3), S2(r) = 1/|C_r| sum_{h in C_r} 2 (R_0 - R_h), C_r = lags
 *     (minimum image, components in {-n/2+1..n/2}) whose length rounds to r;
 *   ek_dev[n/2+1]: energy spectrum E(kappa), kappa = 0..n/2, eq.
 *     (energySpecDisc) with the coefficients of eq. (dftCoeff); modes whose
 *     length rounds above n/2 are not counted.
 * Either output may be NULL. work_dev: device scratch of
 * mclbm_observables_work_bytes(ctx, sample) bytes (about 27 n^3 bytes),
 * 256-byte aligned, owned by the caller. Supported n: 8..512 (a sample
 * of n = 1024 gives MCLBM_ERR_UNSUPPORTED and 0 work bytes). Lattice
 * units (divide by u0^2 for physical units). */
size_t mclbm_observables_work_bytes(const mclbm_ctx* ctx, int32_t sample);
mclbm_status mclbm_observables(mclbm_ctx* ctx, int32_t sample, double* s2_dev, double* ek_dev, void* work_dev,
                               size_t work_bytes);

/* The same for `count` consecutive samples first..first+count-1 that share
 * one n, in one set of launches per run of equal AA parity (the ensemble's
 * resolution groups): s2_dev[count][n/2], ek_dev[count][n/2+1] (device,
 * either may be NULL); work_dev: mclbm_observables_range_work_bytes bytes,
 * 256-byte aligned (0 bytes means an invalid range). MCLBM_ERR_ARG when the
 * range leaves the ensemble or mixes resolutions. */
size_t mclbm_observables_range_work_bytes(const mclbm_ctx* ctx, int32_t first, int32_t count);
mclbm_status mclbm_observables_range(mclbm_ctx* ctx, int32_t first, int32_t count, double* s2_dev, double* ek_dev,
                                     void* work_dev, size_t work_bytes);

/* Velocity capture: the record ticks of mclbm_step read every population of
 * every sample (they fall on ticks where every sample steps), so while a
 * capture buffer is set each record tick also writes the velocity of the
 * state it reads -- the state its record describes -- in double, summed
 * from the populations as eq. (momentDefin) defines it, exactly as the first
 * pass of mclbm_observables_range computes it (the two fields are bitwise
 * equal). Layout: u_dev[voff(s) + a n_s^3 + cell], a = 0, 1, 2 the
 * component, cell = (z n + y) n + x, voff(s) = 3 sum_{s' < s} n_s'^3;
 * mclbm_velocity_bytes(ctx) bytes in total (24 bytes per node). Setting it
 * adds 24 bytes of writes per node to each record tick and lets the
 * observables read 24 bytes per node instead of the populations.
 * mclbm_capture_velocity: u_dev device, 256-byte aligned, at least
 * mclbm_velocity_bytes bytes (else MCLBM_ERR_OOM), owned by the caller, who
 * keeps it alive until the capture is cleared (u_dev NULL) or the context
 * is destroyed; the kernels write it on the context's stream. */
size_t mclbm_velocity_bytes(const mclbm_ctx* ctx);
mclbm_status mclbm_capture_velocity(mclbm_ctx* ctx, double* u_dev, size_t bytes);

/* The observables of mclbm_observables_range (same outputs, work buffer and
 * errors) of the velocity fields held in u_dev (the layout above, e.g. as
 * captured by the last record tick), for samples first..first+count-1 that
 * share one n, in one set of launches. u_dev: device, 256-byte aligned,
 * read only, holding at least the planes of those samples at their offsets
 * (mclbm_velocity_bytes(ctx) bytes for the whole layout; the library cannot
 * check the length of a raw pointer); the state of the ensemble is not
 * read. */
mclbm_status mclbm_observables_velocity_range(mclbm_ctx* ctx, int32_t first, int32_t count, const double* u_dev,
                                              double* s2_dev, double* ek_dev, void* work_dev, size_t work_bytes);

/* Sample-wise compensation (eqs. (compensatedE), (compensatedSF)) of the
 * observables of samples first..first+count-1, which share one n:
 * ekc_dev[s][kappa] = kappa^(5/3) (E_s(kappa) / u0_s^2) / (C_Kol d_s^(2/3)),
 * C_Kol = 1.5, and s2c_dev[s][r-1] = (S2_s(r) / u0_s^2) / (d_s r 2 pi / n)^(2/3)
 * for the lag r = 1..n/2 (physical lag r 2 pi / n), with d^(2/3) taken as
 * the cube root of d^2 and d_s the sample's dissipation rate at the time of
 * the observables (diss_dev[count], device: a row of mclbm_dissipation's
 * output from sample `first` on). s2_dev, s2c_dev: [count][n/2]; ek_dev,
 * ekc_dev: [count][n/2 + 1] (device, double, as written by
 * mclbm_observables_range); either pair may be NULL, not half of one. The
 * inner-scaled abscissae are kappa eta and r 2 pi / (n eta) with eta from
 * mclbm_dissipation. Runs on the context's stream. MCLBM_ERR_ARG (nothing
 * enqueued) for a range outside the ensemble, samples of different n, a NULL
 * diss_dev or half a pair; both pairs NULL is a no-op. */
mclbm_status mclbm_compensate(mclbm_ctx* ctx, int32_t first, int32_t count, const double* diss_dev,
                              const double* s2_dev, const double* ek_dev, double* s2c_dev, double* ekc_dev);

/* Velocity of every sample at the q^3 nodes common to all resolutions
 * (node j = (jx, jy, jz) at lattice index (n/q) j, i.e. x = 2 pi j / q):
 * out_dev[m][3][q^3], double, component-major per sample (appendix on the
 * Wasserstein distances: exact restriction to the common downsampled grid).
 * physical = 1 gives u / u0 (velocities of different resolutions in the
 * same units), 0 lattice units. q must divide every sample's n. */
mclbm_status mclbm_point_values(mclbm_ctx* ctx, int32_t q, int32_t physical, double* out_dev);

/* 1-point Wasserstein distance W_{1,1} between two ensembles (Algorithm 2 with
 * eq. (wassersteinPermutations)): for each node and component, W1 of the two
 * empirical laws of m equal-weight values (sorted rearrangement), summed over
 * the q^3 nodes and divided by q^3. a_dev, b_dev: point values
 * [m][3][q^3] (as written by mclbm_point_values); out_dev[3] receives the
 * per-component terms D_c / q^3 (their sum is W_{1,1}). m <= 4096, q <= 64.
 * work_dev: mclbm_w1_work_bytes(q) bytes of device scratch. Runs on
 * hip_stream. */
size_t mclbm_w1_work_bytes(int32_t q);
mclbm_status mclbm_w1_1pt(const double* a_dev, const double* b_dev, int32_t m, int32_t q, double* out_dev,
                          void* work_dev, size_t work_bytes, void* hip_stream);

/* Empirical ensemble statistics (eqs. (spectrum_mean), (spectrum_var)): for
 * each column c < k of x_dev[m][ld] (device, double, rows of ld >= k values),
 * mean_dev[c] = (1/m) sum_i x[i][c] and std_dev[c] = sqrt(1/(m-1) sum_i
 * (x[i][c] - mean_dev[c])^2), in two fixed-order FP64 passes on hip_stream.
 * std_dev may be NULL (then m >= 1; with it m >= 2, else MCLBM_ERR_ARG).
 * Rows of samples: the spectra or structure functions of a resolution group
 * (ld = n/2 + 1 or n/2), or KE of one record (x_dev = records + 4, ld = 8). */
mclbm_status mclbm_ensemble_moments(const double* x_dev, int32_t m, int32_t k, int64_t ld, double* mean_dev,
                                    double* std_dev, void* hip_stream);

/* Ensemble-mean relative L1 distance between the samples of two ensembles at
 * the common nodes (eq. (sample_error)): out_dev[k] = (1/m) sum_m
 * sum_nodes |a_m - b_m| / sum_nodes |b_m|, with b the reference ensemble and
 * sample m of both drawn from the same Y_m; k = 0, 1, 2 take |.| of one
 * velocity component, k = 3 the Euclidean length of the velocity vector.
 * a_dev, b_dev: point values [m][3][q^3] (device, double, as written by
 * mclbm_point_values); out_dev[4] (device). A sample whose reference values
 * of a quantity are all zero, where the definition has no value, makes that
 * quantity +inf (NaN if its own values are all zero too). 1 <= m <= 2^20,
 * 1 <= q <= 64. work_dev: mclbm_sample_error_work_bytes(m) bytes of device
 * scratch. Runs on hip_stream; the result does not depend on the launch
 * (fixed summation order). */
size_t mclbm_sample_error_work_bytes(int32_t m);
mclbm_status mclbm_sample_error(const double* a_dev, const double* b_dev, int32_t m, int32_t q, double* out_dev,
                                void* work_dev, size_t work_bytes, void* hip_stream);

/* mclbm_sample_error without a caller-provided work buffer, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result, bit for bit, with the per-sample partial ratios in a device array
 * of the library (4 doubles per sample, 2 MiB: m <= 65536, else
 * MCLBM_ERR_ARG before anything is enqueued). Each GPU holds its own copy of
 * that array until the process ends; the call allocates nothing. Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be ordered by
 * the caller. Runs on hip_stream, which must belong to the current device. */
mclbm_status mclbm_sample_error_noalloc(const double* a_dev, const double* b_dev, int32_t m, int32_t q,
                                        double* out_dev, void* hip_stream);

/* Experimental order of convergence (Algorithm (ComputeSlopes)): the slope
 * of the least-squares line through (log n[i], log d[i]), i < k, where d[i]
 * is a distance of resolution n[i] to the reference resolution (host
 * arrays; k >= 2; all values positive and finite; not all n equal, else
 * MCLBM_ERR_ARG). *slope (host) receives it. Host only: no device call. */
mclbm_status mclbm_eoc_slope(const double* n, const double* d, int32_t k, double* slope);

/* Dissipation rate per unit volume and Kolmogorov length from a series of
 * records of mclbm_step. The paper defines the sample dissipation rate
 * (before eq. (kolmogorov_microscale)) as nu ||grad u_m||^2 / |Omega| and
 * approximates it by the decay of the energy per unit volume; this call
 * differentiates the kinetic energy per unit volume of the records:
 * d_m(t) = -(d/dt) KE_m(t), with KE_m in units of u0^2 (field 4 of the
 * records divided by u0^2; the Parseval sum over every mode) and t the
 * physical time of the record, t = steps * (2 pi / n) * u0 (unit reference
 * velocity, box of side 2 pi); the derivative is a centred difference
 * inside the series and one-sided at its ends. The paper's own
 * approximation differentiates the summed shell spectrum instead
 * (mclbm_dissipation_spectra); the two differ by the shell weights of eq.
 * (energySpecDisc) (a factor 4 pi 3 / 62 = 0.61 for energy in the Taylor-
 * Green modes, tending to 1 as the energy moves to high shells).
 * eta(t) = (eps^3 / mean_m d_m(t))^(1/4) with eps = 1 / Re, eq.
 * (kolmogorov_microscale).
 * records_dev: [nrec][m][8] (device) as written by mclbm_step, the first
 * taken at tick first_tick, the others every record_every ticks (both
 * multiples of every stride; nrec >= 2). diss_dev: [nrec][m] (device).
 * eta_dev: [nrec] (device) or NULL; it needs one Re for all samples
 * (MCLBM_ERR_ARG otherwise); a non-positive mean dissipation gives NaN. */
mclbm_status mclbm_dissipation(mclbm_ctx* ctx, const double* records_dev, int32_t nrec, int64_t first_tick,
                               int32_t record_every, double* diss_dev, double* eta_dev);

/* The paper's approximation of the sample dissipation rate (the sentence
 * after its definition, before eq. (kolmogorov_microscale)):
 * d_m(t) = -(d/dt) sum_kappa E_m(kappa, t), with E_m the shell spectrum of
 * eq. (energySpecDisc) in units of u0^2, for the `count` samples
 * first..first+count-1 of one resolution, from their spectra at nrec saved
 * times: ek_dev[nrec][count][n/2+1] (device, lattice units, each row as
 * written by mclbm_observables_range), the first saved at tick first_tick,
 * the others every record_every ticks (multiples of the samples' stride).
 * Time, differences and eta as in mclbm_dissipation; diss_dev[nrec][count]
 * (device); eta_dev[nrec] (device) or NULL, from the mean over the range
 * (one Re for the range, else MCLBM_ERR_ARG). MCLBM_ERR_ARG (nothing
 * enqueued) for a range outside the ensemble or of mixed resolutions,
 * nrec < 2, or saved ticks where a sample of the range does not step. */
mclbm_status mclbm_dissipation_spectra(mclbm_ctx* ctx, int32_t first, int32_t count, const double* ek_dev,
                                       int32_t nrec, int64_t first_tick, int32_t record_every, double* diss_dev,
                                       double* eta_dev);

/* Stabiliser gamma of the higher-order relaxation omega_hom = omega gamma / 2
 * (Table 1). MCLBM_GAMMA_CLOSED_FORM (default) evaluates eq. (entropyControl).
 * MCLBM_GAMMA_EXACT minimises the discrete H-function of the post-collision
 * state, eq. (kbc_entropy): with t = omega gamma / 2, H(t) is convex where
 * every f*_i > 0; safeguarded Newton steps on H'(t) = 0 start from the
 * closed form (a step leaving that interval is replaced by the midpoint
 * towards its edge) and stop, per node, once a step is below 2^-12 of t in
 * FP32 or 1e-8 in FP64 (at most four), so the records report the exact
 * gamma. The exact mode
 * runs 256-thread blocks only (mclbm_set_launch accepts no other size then,
 * mclbm_autotune returns MCLBM_ERR_UNSUPPORTED); mclbm_forward_ckpt and
 * mclbm_backward differentiate it in FP64. Captured graphs are dropped.
 * MCLBM_ERR_ARG for any other mode. */
mclbm_status mclbm_set_stabiliser(mclbm_ctx* ctx, int32_t mode);

/* Launch shape of the collide-and-stream kernel, one for the whole ensemble
 * launch: threads (= lattice nodes) per block, 128, 256, 512 or 1024 (1024:
 * FP32 only), not above any sample's n^3; xcd_remap = 1 renumbers blocks so
 * that each of the 8 XCDs works on one contiguous range of nodes;
 * buffer_addressing = 1 addresses the population planes through one buffer
 * resource per sample (scalar plane offsets, 32-bit lane offsets), used only
 * while every sample's populations span less than 2 GiB, else plain 64-bit
 * pointers; nontemporal = 1 marks the population loads and stores
 * non-temporal. None of these changes a result. Invalidates cached graphs. */
mclbm_status mclbm_set_launch(mclbm_ctx* ctx, int32_t block_threads, int32_t xcd_remap, int32_t buffer_addressing,
                              int32_t nontemporal);
mclbm_status mclbm_get_launch(const mclbm_ctx* ctx, int32_t* block_threads, int32_t* xcd_remap,
                              int32_t* buffer_addressing, int32_t* nontemporal);

/* Time every launch shape on the current state (`reps` periods of
 * 2 * max stride ticks each, after one warm-up period), time the three
 * fastest twice more, keep the one with the best time,
 * and restore the state from a checkpoint written to scratch_dev
 * (mclbm_checkpoint_bytes). best_* (may be NULL) receive the choice. On an
 * error the launch shape and the state are put back as they were and the
 * error of the failing trial is returned. */
mclbm_status mclbm_autotune(mclbm_ctx* ctx, int32_t reps, void* scratch_dev, size_t scratch_bytes,
                            int32_t* best_block, int32_t* best_xcd, int32_t* best_buffer, int32_t* best_nt);

/* Capture the tick loop into HIP graphs (1, the default) or launch kernel by
 * kernel (0). Graphs are used only on a non-NULL stream, for runs of at
 * least one graph length (a whole number of activity/parity periods). */
mclbm_status mclbm_use_graphs(mclbm_ctx* ctx, int32_t enable);

/* Current tick counter and the number of steps sample s has taken. */
int64_t mclbm_ticks(const mclbm_ctx* ctx);
int64_t mclbm_steps(const mclbm_ctx* ctx, int32_t sample);

/* Average duration in milliseconds, measured with HIP events on the
 * context's stream, of the collide-and-stream launches enqueued since the
 * last call (timing must be switched on with mclbm_time_launches(ctx, 1);
 * it brackets every tick launch with events and switches graphs off while
 * on). *launches gets the count. The context keeps two events per timed
 * launch until mclbm_launch_time reads them, and reuses them afterwards. */
mclbm_status mclbm_time_launches(mclbm_ctx* ctx, int32_t enable);
mclbm_status mclbm_launch_time(mclbm_ctx* ctx, double* avg_ms, int64_t* launches);

/* Device-to-device copy of `bytes` (a multiple of 16) with a plain vector
 * copy kernel (one 16-byte non-temporal load and store per thread) on
 * `hip_stream`: the measured HBM bandwidth reference. */
mclbm_status mclbm_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream);

/* Message of the last failing call on this thread ("" if none). */
const char* mclbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCLBM_H */
