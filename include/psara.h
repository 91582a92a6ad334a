/*
 * psara.h -- C ABI of the MI355X (gfx950) Polarized SARA library.
 *
 * Polarized SARA (Birdi, Repetti & Wiaux, MNRAS 2018) images the four Stokes
 * maps S = [I, Q, U, V] in R^{N x 4} from full-polarisation visibilities
 * Y in C^{M x 4} by solving (eq. min_gen2)
 *
 *   minimise  iota_B(Y,eps)(phi(S)) + iota_U(S) + gamma ||Psi^dagger S||_{W,1}
 *             + iota_V(Z) + iota_E1(S_:1, Z_:1) + iota_E2(S_:2:4, Z_:2)
 *
 * with the primal-dual iteration of Algorithm 1 (Sec. 3.3) inside the
 * reweighting loop of Algorithm 2 (Sec. 3.3.4).  The library owns all device
 * state of one solve in an opaque context; every step of the iteration runs in
 * hand-written HIP kernels.  Host arrays passed in are caller-owned and copied
 * before the call returns; nothing is retained.  All calls are synchronous with
 * respect to the host unless stated otherwise, and return a psara_status; the
 * message of the last failure is available from psara_last_error().
 *
 * Conventions shared by every call:
 *   - images are N x 4 row-major doubles, N = n*n, pixel p = r*n + c (row r,
 *     column c, centred coordinates (r - n/2, c - n/2)), columns I, Q, U, V;
 *   - visibilities are M x 4 complex doubles stored as interleaved (re, im)
 *     pairs, i.e. 8 doubles per row, columns the brightness products
 *     [I+Q, U+iV, U-iV, I-Q] of Sec. 2.1;
 *   - uv points are M x 2 doubles in radians per pixel, each in [-pi, pi),
 *     component 0 pairing with the row axis;
 *   - SARA coefficients are J x 4 doubles, J = nb * N, one n x n block per
 *     basis in the order Dirac, Db1 ... Db8 (bases absent from the mask are
 *     skipped), each block in the in-place Mallat layout of a periodised 2-D
 *     DWT (rows first, then columns, per level).
 *
 * A context is bound to one HIP stream and one device and is not re-entrant;
 * distinct contexts may be used from distinct threads.
 */
#ifndef PSARA_H
#define PSARA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psara_ctx psara_ctx;

typedef enum {
    PSARA_OK = 0,
    PSARA_EINVAL = -1,   /* invalid argument (sizes, ranges, step-size condition) */
    PSARA_ENOMEM = -2,   /* device allocation failed */
    PSARA_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed */
    PSARA_ESTATE = -4,   /* call out of order (e.g. solve before set_data) */
    PSARA_ENAN = -5      /* non-finite input */
} psara_status;

typedef enum {
    PSARA_FP64 = 0,        /* every array and every operation in double precision */
    PSARA_FP32_MIXED = 1   /* FP32 arrays and operators; l2-ball norm, power iteration
                              and stopping reductions in FP64 with compensated sums */
} psara_precision;

typedef enum {
    PSARA_CONSTRAINED = 0,   /* Polarized SARA, eq. min_gen2 (all terms of Algorithm 1) */
    PSARA_NNLS_INIT = 1,     /* initialisation of Sec. 3.3.4: g = 0, set U' (I >= 0); only S, B move */
    PSARA_UNCONSTRAINED = 2  /* "Polarized SARA without constraint", eq. min_gen_matrix_no_flux */
} psara_mode;

/* Stopping and diagnostic quantities of Sec. 4.2 and Sec. 4.6, all FP64. */
typedef struct {
    double residual;     /* ||phi(S) - Y||_2 */
    double epsilon;      /* l2 bound of the data-fidelity ball */
    double rel_var[4];   /* ||S_i^(k) - S_i^(k-1)|| / ||S_i^(k-1)|| per Stokes map (inf if 0 / 0) */
    double zeta;         /* 3 x rms of the Stokes-I residual image Re phi^dagger(Y - phi(S)) / (2M) */
    double n_p;          /* percentage of pixels with ||S_n,2:4|| - S_n,1 > zeta */
    double objective;    /* ||Psi^dagger S||_{W,1} with the current weights */
    double vnorm;        /* ||B~/rho2 - Y|| at the last dual-B step */
    int64_t iterations;  /* Algorithm-1 iterations run on this context so far */
} psara_report;

/* Stopping criteria of Sec. 4.6, tested on the device after every check: a run stops when
 * ||phi(S) - Y|| <= (1 + theta) epsilon, the largest relative variation of the four Stokes maps
 * between the last two iterates is <= rel_var (a map that is zero in both counts as 0), and,
 * when np_max >= 0, N_p <= np_max (percent).  The paper's setting: theta = 5e-3,
 * rel_var = 1e-5, np_max = 0.5 for the constrained problem (np_max < 0 disables the test). */
typedef struct {
    double theta;
    double rel_var;
    double np_max;
} psara_stop;

/* ---- lifetime --------------------------------------------------------------------------- */

/* Create a context on `device`.  `hip_stream` is a hipStream_t to run on (for example
 * torch.cuda.current_stream().cuda_stream) or NULL for a library-owned stream.  PSARA_EDEVICE
 * when no device is present or when psara_runtime_check fails. */
psara_status psara_create(psara_ctx** out, int device, void* hip_stream);
void psara_destroy(psara_ctx* ctx);
const char* psara_last_error(const psara_ctx* ctx);
const char* psara_status_string(psara_status s);

/* Checks that the HIP runtime the process runs on has the major and minor version the library
 * was built against: a process that has loaded another HIP runtime first (for example the one a
 * Python framework bundles) makes the library run on that one, whose types and entry points need
 * not match.  built / running (may be NULL) receive the two versions as major * 10^7 +
 * minor * 10^5 + patch (running 0 if the runtime cannot be queried).  PSARA_OK when they
 * agree, PSARA_EDEVICE otherwise.  psara_create and psara_server_create refuse to start on a
 * mismatch.  Needs no device. */
psara_status psara_runtime_check(int* built, int* running);

/* ---- problem set-up (Sec. 2.2, 3.1, 4.1) --------------------------------------------------- */

/* Measurement operator phi = G F Z . L (eq. meas_op): n x n images (n a power of two,
 * 8 <= n <= 1024), M >= 1 uv points (copied; sorted into grid tiles on the device side),
 * oversampling 2 per dimension, Kaiser-Bessel interpolation with `taps` in {4, 6, 8} per
 * dimension.  Resets data, prior, steps and state.  EINVAL on bad sizes or uv outside
 * [-pi, pi). */
psara_status psara_set_operator(psara_ctx* ctx, int n, int64_t M, const double* uv,
                                int oversample, int taps, psara_precision precision);

/* Visibilities Y (M x 4 complex, see conventions) and the l2 bound epsilon > 0 of the
 * data-fidelity ball B(Y, epsilon) (eq. f_diff).  ENAN if Y holds a non-finite value. */
psara_status psara_set_data(psara_ctx* ctx, const double* Y, double epsilon);

/* psara_set_data with Y in device memory of the context's device (borrowed for the call only:
 * the call returns once the library no longer reads it; the caller must have finished writing
 * it, since the call is not ordered after the caller's streams).  Same layout and checks
 * (ENAN, Y unchanged, if a value is not finite); the row permutation and the conversion to the
 * working precision run on the device.  EINVAL for NULL or a pointer that is not device or
 * managed memory of the context's device. */
psara_status psara_set_data_dev(psara_ctx* ctx, const double* Y, double epsilon);

/* SARA prior (Sec. 3.1): basis_mask bit 0 = Dirac, bits 1..8 = Db1..Db8; `levels` >= 1 with
 * n divisible by 2^levels; weights W (J x 4, >= 0) or NULL for all ones; gamma > 0 (the free
 * scale of eq. min_gen2).  The soft-threshold sizes are gamma * W.  Psi is normalised by
 * 1/sqrt(nb) so that Psi Psi^dagger = I. */
psara_status psara_set_prior(psara_ctx* ctx, uint32_t basis_mask, int levels,
                             const double* weights, double gamma);

/* Step sizes of Algorithm 1.  EINVAL unless all are > 0 and the convergence condition of
 * Sec. 3.3.3,  1/tau - rho1 ||Psi||^2 - rho2 ||phi||^2 - rho3 >= 0,  holds with the
 * operator norm from psara_opnorm (which must have run). */
psara_status psara_set_steps(psara_ctx* ctx, double tau, double rho1, double rho2, double rho3);

/* Step sizes meeting that condition (Sec. 3.3.3 gives only the condition; the values are this
 * library's choice): prior 0 (SARA, ||Psi|| = 1, Algorithm 1): rho1 = rho3 = 1,
 * rho2 = 1 / ||phi||^2, tau = margin / (rho1 + rho2 ||phi||^2 + rho3) = margin / 3; prior 1 (TV)
 * or 2 (l1 + TV) of Algorithm 3: rho1 = 1 / ||Psi||^2 with ||Psi||^2 = 8 or 9, rho2 = 1 (unused),
 * rho3 = 1, tau = margin / (||phi||^2 / 4 + rho1 ||Psi||^2 + rho3).  phi_norm_sq > 0,
 * 0 < margin <= 1 (0.99 keeps a 1 % margin from the bound).  out: tau, rho1, rho2, rho3.
 * Needs no device. */
psara_status psara_step_sizes(int prior, double phi_norm_sq, double margin, double* out);

/* psara_set_steps with the values of psara_step_sizes for the context's prior and the operator
 * norm of its last psara_opnorm; out (NULL or 4 doubles) receives them. */
psara_status psara_set_steps_auto(psara_ctx* ctx, double margin, double* out);

/* The TV-based priors of Sec. 4.3 instead of SARA: the context then runs Algorithm 3 for
 * eq. Akiyama_2 (PSARA_CONSTRAINED: with the polarization constraint) or eq. Akiyama
 * (PSARA_UNCONSTRAINED: I >= 0 only), whose data term is 1/2 ||Y L^{-1} - phi~(S)||^2 with
 * phi~ = phi without the mixing L (the data are those of psara_set_data, in brightness order).
 * l1 = 0: TV, g = sum_i tv_weight[i] ||grad S_i||_{2,1}; l1 = 1: l1 + TV, adding
 * sum_i l1_weight[i] ||S_i||_1.  grad: forward differences along both image axes with a zero
 * difference at the last row and column.  The dual A (psara_get_state) is then 2N x 4 (the d1
 * block, the d2 block) or 3N x 4 for l1 + TV (the Dirac block first).  Weights finite and > 0.
 * Step sizes (again
 * through psara_set_steps, rho2 unused but > 0) must satisfy
 * 1/tau - rho1 ||Psi||^2 - rho3 >= ||phi||^2 / 4 with ||Psi||^2 = 8 (TV) or 9 (l1 + TV)
 * (||phi~||^2 = ||phi||^2 / 2 is the Lipschitz constant of the data term's gradient).  The
 * reweighting, the initialisation mode, batches, the server and Mueller matrices are defined
 * for the SARA prior only (PSARA_EINVAL).  The iterations start from the current state. */
psara_status psara_set_prior_tv(psara_ctx* ctx, int l1, const double* tv_weight, const double* l1_weight);

/* Known direction-independent Mueller matrices (eq. RIME with D_m not depending on the sky
 * position): row m of the visibilities becomes y_m = D_m (S^T L)^T evaluated at u_m, i.e. the
 * fixed brightness mixing L is replaced per row by L D_m^T, in phi and in its adjoint.  D: M
 * row-major 4 x 4 complex matrices, interleaved (re, im), in the caller's visibility order
 * (copied); D_m acts on the brightness vector [I+Q, U+iV, U-iV, I-Q].  NULL restores L.  The
 * iteration state is reset, and psara_opnorm and psara_set_steps must be called again. */
psara_status psara_set_mueller(psara_ctx* ctx, const double* D);

/* ||phi||^2 of the real-restricted map S -> Re phi^dagger phi S by an FP64 power
 * iteration on the device (seeded start), stopped when the Rayleigh quotient changes by
 * less than rtol (relative) or after max_iter iterations.  Stored in the context. */
psara_status psara_opnorm(psara_ctx* ctx, int max_iter, double rtol, double* phi_norm_sq);

/* ---- the iteration (Algorithm 1) and the reweighting (Algorithm 2) ------------------------- */

/* Run `iters` iterations of Algorithm 1 in `mode` from the current state (warm start, as
 * Algorithm 2 passes every variable from one reweighting cycle to the next).  Iterations
 * are replayed from a captured HIP graph.  If `check_every` > 0 the stopping quantities are
 * evaluated every check_every iterations; if `out` is not NULL it receives the quantities
 * after the last iteration. */
psara_status psara_solve(psara_ctx* ctx, psara_mode mode, int iters, int check_every,
                         psara_report* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * that forbid allocation): psara_solve(ctx, mode, iters, 0, NULL) by direct kernel launches
 * (no graph is captured or instantiated), with the iteration's scratch buffers -- the gridding
 * partial slots and the FP64 partial sums -- in a static device array of the library (32 MiB,
 * held on every device the library runs on until the process ends) instead of the context's
 * own; no device memory is allocated or freed.  The resulting state is bit for bit that of
 * psara_solve.  PSARA_EINVAL when the problem needs more scratch than the array holds (the
 * slots take (16 + taps - 1)^2 cells of 8 reals per gridding chunk: about 14 MiB for a 256 x 256
 * image with 2e5 rows in FP32, twice that in FP64).  Every call on one device shares that
 * device's array: calls that overlap on one device (from several threads, or on several
 * contexts' streams at once) race.  Blocks until the iterations are done. */
psara_status psara_solve_noalloc(psara_ctx* ctx, psara_mode mode, int iters);

/* Capture, without running anything, the HIP graphs that psara_solve(ctx, mode, iters,
 * check_every, ...) replays; a solve captures the graphs it lacks itself, so this only moves
 * that work ahead of a timed or latency-critical call.  A solve of `iters` iterations replays
 * chains of 32 captured iterations and one chain of the remainder.  Requirements as for
 * psara_solve. */
psara_status psara_capture(psara_ctx* ctx, psara_mode mode, int iters, int check_every);

/* Run Algorithm 1 in `mode` from the current state until the criteria `stop` hold or
 * max_iters iterations have run.  The criteria are evaluated on the device (FP64 reductions)
 * after every check_every iterations (check_every >= 1), inside the captured graph; the host
 * reads the outcome one check behind without waiting for the work it has just queued, and
 * checks queued after the stop do nothing.  The iterations run are added to the context's
 * count (out->iterations) and written to *iters_run if it is not NULL.  stop->theta >= 0,
 * stop->rel_var >= 0. */
psara_status psara_solve_adaptive(psara_ctx* ctx, psara_mode mode, int max_iters, int check_every,
                                  const psara_stop* stop, int* iters_run, psara_report* out);

/* Algorithm 2 with adaptive stages: the initialisation stage and every reweighted stage run
 * as psara_solve_adaptive with at most max_iters_per_stage iterations; the initialisation
 * stage uses the residual and relative-variation tests only (N_p is not part of its problem).
 * iters_run: NULL or cycles + 1 counts, the iterations each stage ran. */
psara_status psara_reweighted_solve_adaptive(psara_ctx* ctx, psara_mode mode, int cycles,
                                             int max_iters_per_stage, int check_every,
                                             const psara_stop* stop, double delta_decay,
                                             int* iters_run, psara_report* out);

/* Reweighting step of Algorithm 2 (eq. weights): W = delta / (delta + |Psi^dagger S|),
 * thresholds gamma * W.  delta > 0. */
psara_status psara_reweight(psara_ctx* ctx, double delta);

/* Standard deviation of the 4J entries of Psi^dagger S (FP64), the starting delta of the
 * reweighting schedule. */
psara_status psara_coef_std(psara_ctx* ctx, double* out);

/* Algorithm 2 end to end: an initialisation stage (PSARA_NNLS_INIT) of iters_per_stage[0]
 * iterations, then `cycles` reweighted stages in `mode` of iters_per_stage[1..cycles]
 * iterations each; delta starts at the coefficient standard deviation after the
 * initialisation and is divided by delta_decay (> 1) after every cycle. */
psara_status psara_reweighted_solve(psara_ctx* ctx, psara_mode mode, int cycles,
                                    const int* iters_per_stage, double delta_decay,
                                    psara_report* out);

/* Evaluate the stopping quantities for the current state. */
psara_status psara_report_now(psara_ctx* ctx, psara_report* out);

/* Wait until all work queued on the context's stream has finished (psara_solve and the other
 * iteration calls return once their launches are queued).  EDEVICE if the device reports an
 * error for that work. */
psara_status psara_synchronize(psara_ctx* ctx);

/* The data-driven regularisation weight gamma = factor * ||Psi^dagger Re phi^dagger Y||_inf /
 * ||phi||^2 (the choice of gamma used with the paper's setting, factor 1e-3), computed on the
 * device.  Requires operator, data, prior and psara_opnorm.  Does not change the context. */
psara_status psara_data_gamma(psara_ctx* ctx, double factor, double* gamma);

/* Replace gamma in the thresholds gamma W of the prior (W unchanged); gamma > 0. */
psara_status psara_set_gamma(psara_ctx* ctx, double gamma);

/* ---- launch shapes and the autotuner ----------------------------------------------------- */

/* Launch shapes of a solve.  They change how the work is cut into workgroups and so the
 * summation order of the gridding and of the de-gridding norm (results differ at rounding level,
 * never in what is computed); every solve starts with the defaults. */
typedef struct {
    int grid_chunk;      /* gridding entries per workgroup: 256, 512 or 1024 (default 1024) */
    int degrid_item;     /* visibilities per de-gridding workgroup: a power of two in [64, 1024]
                            (default 256) */
    int analysis_wide;   /* bit 0: 16-wide output tiles for the analysis bands of side >= 128 of
                            FP32 solves (else 8-wide: more workgroups); bit 1: each level-1
                            workgroup of the iterations filters one staged image region with every
                            wavelet basis (the region is staged once, not once per basis);
                            0 .. 3, default 1 */
    int fft_cells;       /* grid cells per FFT workgroup: 0 for max(512, 2n) (default), or 512, 1024,
                            2048 with at least 2n (several grid lines per workgroup) */
} psara_tuning;

/* The context's launch shapes (ESTATE before psara_set_operator). */
psara_status psara_get_tuning(const psara_ctx* ctx, psara_tuning* out);
/* Apply launch shapes (NULL: the defaults): the gridding lists are cut again and the work lists
 * rebuilt; the iteration state is kept.  EINVAL outside the ranges above. */
psara_status psara_set_tuning(psara_ctx* ctx, const psara_tuning* t);

enum {
    PSARA_TUNE_USE_CACHE = 1,   /* take the shapes stored for this shape class, if any, without timing */
    PSARA_TUNE_STORE = 2        /* store the chosen shapes for the class (process-wide) */
};

/* The autotuner: times the iteration of `mode` (chains of 8 captured iterations, best of three)
 * under candidate shapes, one parameter at a time from the current ones (grid_chunk 1024 / 512 /
 * 256, degrid_item 256 / 128 / 512, analysis_wide 1 / 0 / 3 / 2, fft_cells default / 1024 / 2048), keeps
 * a candidate that beats the incumbent by 1 %, and applies the fastest.  The iteration state is
 * saved and restored around the trials (the stored state exactly; the operator images the next
 * primal step reads are recomputed).  A shape class is the precision, taps, image side, levels,
 * basis mask and the visibility count's power of two.  flags: PSARA_TUNE_USE_CACHE,
 * PSARA_TUNE_STORE.  chosen: NULL or the shapes applied; ms_per_iter: NULL or 2 doubles, the
 * iteration time of the starting shapes and of the chosen ones (0, 0 for a cache hit).
 * Requirements as for psara_solve in `mode`. */
psara_status psara_autotune(psara_ctx* ctx, psara_mode mode, int flags, psara_tuning* chosen, double* ms_per_iter);

/* The autotuner for a batch (the requirements of psara_batch_solve): every candidate is applied
 * to all members and timed as one batched iteration; the chosen shapes end up applied to every
 * member.  Not stored per class. */
psara_status psara_batch_autotune(psara_ctx* const* ctxs, int count, psara_mode mode, psara_tuning* chosen,
                                  double* ms_per_iter);

/* The shapes stored for a shape class by psara_autotune with PSARA_TUNE_STORE: PSARA_OK and
 * *out, or PSARA_ESTATE when none is stored.  Needs no device. */
psara_status psara_tuning_lookup(int n, int64_t M, int taps, int levels, uint32_t basis_mask,
                                 psara_precision precision, psara_tuning* out);

/* ---- batches of independent solves ------------------------------------------------------- */

/* Advance `count` independent solves together: every pass of Algorithm 1 is one launch over
 * all of them (their work lists concatenated), captured in one HIP graph on the stream of
 * ctxs[0]; each solve keeps its own state and its result is the same as when it runs alone
 * (the kernels' arithmetic per problem does not depend on the batch).  Requirements: count >= 1
 * distinct contexts on one device with the same precision and tap count, each with operator,
 * data and step sizes set, and a prior for the modes with the sparsity term.  Blocks until the
 * iterations are done.  reports: NULL or `count` reports filled as psara_solve does.  On an
 * error every context's last error holds the message and no iteration has run. */
psara_status psara_batch_solve(psara_ctx* const* ctxs, int count, psara_mode mode, int iters,
                               psara_report* reports);

/* Algorithm 2 for a batch: the initialisation stage batched, then for each member its own
 * delta (coefficient standard deviation) and weights, then `cycles` batched reweighted stages,
 * delta divided by delta_decay after every cycle, exactly as psara_reweighted_solve per member.
 * reports: NULL or `count` final reports. */
psara_status psara_batch_reweighted_solve(psara_ctx* const* ctxs, int count, psara_mode mode, int cycles,
                                          const int* iters_per_stage, double delta_decay,
                                          psara_report* reports);

/* ---- state ------------------------------------------------------------------------------- */

/* Current Stokes estimate S (N x 4 doubles). */
psara_status psara_get_image(psara_ctx* ctx, double* S);
/* psara_get_image into device memory of the context's device (N x 4 doubles, same layout;
 * returns once written).  EINVAL for NULL or a pointer that is not device or managed memory of
 * the context's device. */
psara_status psara_get_image_dev(psara_ctx* ctx, double* S);

/* Size in bytes of the serialised state: (N*4 + N*2 + J*4 + M*8 + N*4 + N*2) doubles holding
 * S, Z, A, B (complex, original uv order), C, D in that order. */
size_t psara_state_bytes(const psara_ctx* ctx);
psara_status psara_get_state(psara_ctx* ctx, void* buf, size_t bytes);
psara_status psara_set_state(psara_ctx* ctx, const void* buf, size_t bytes);
/* All primal and dual variables to zero (Algorithm 1's starting point used here). */
psara_status psara_reset_state(psara_ctx* ctx);

/* Device bytes a context of this shape allocates (used for admission control). */
size_t psara_footprint(int n, int64_t M, int taps, int levels, uint32_t basis_mask,
                       psara_precision precision);

/* ---- operators (for verification and synthetic data; same kernels as the iteration) ------ */

/* Y = phi(S) (eq. meas_op): S is N x 4, Y is M x 4 complex in the caller's uv order. */
psara_status psara_apply_phi(psara_ctx* ctx, const double* S, double* Y);
/* S = Re phi^dagger(B) (the adjoint followed by the projection onto real matrices). */
psara_status psara_apply_phi_adjoint(psara_ctx* ctx, const double* B, double* S);
/* A = Psi^dagger S (J x 4) and S = Psi A, for the prior set by psara_set_prior. */
psara_status psara_apply_psi_adjoint(psara_ctx* ctx, const double* S, double* A);
psara_status psara_apply_psi(psara_ctx* ctx, const double* A, double* S);

/* ---- host-only helpers (no device needed) ------------------------------------------------ */

/* Daubechies low-pass filter with p in [1, 8] vanishing moments by spectral factorisation
 * (minimum phase); writes 2p doubles.  Returns 2p, or 0 on bad p. */
int psara_wavelet_filter(int p, double* h);

/* Kaiser-Bessel shape beta for `taps` and oversampling alpha (Beatty et al. 2005) and the
 * kernel value psi(t) / deapodisation 1/psi_hat(nu) used by the operator. */
double psara_kb_beta(int taps, double alpha);
double psara_kb_value(int taps, double beta, double t);
double psara_kb_deapod(int taps, double beta, double nu);

/* Sorted-visibility layout chosen by set_operator: writes the permutation (sorted position
 * -> caller index, M entries) and returns the grid tile side, or a negative status. */
int psara_layout(const psara_ctx* ctx, int64_t* perm);

/* ---- profiling --------------------------------------------------------------------------- */

/* Run `iters` iterations of Algorithm 1 in `mode` with every launch on the context stream
 * (no graph, the two independent branches serialised), bracket each pass with HIP events,
 * and write the average duration in milliseconds of each pass to ms_per_pass[0..8]:
 * [0] primal / epigraph / Dirac dual step fused with the zero-padding and row FFT (P1+P4),
 * [1] SARA analysis + dual A + synthesis (P2+P3, coarse levels fused), [2] and [3] zero (their
 * work is timed in [1] and [0]), [4] column FFT (P5), [5] de-grid + dual B (P6), [6] grid (P7),
 * [7] column inverse FFT (P8, which also sums the partial tiles of split gridding tiles),
 * [8] row inverse FFT + crop (P9), then runs `iters` more iterations in the order the captured
 * graphs use and writes to ms_per_pass[9] the average duration of the pass that fuses P9 with
 * the next iteration's P1+P4 (0 when iters < 2) and to ms_per_pass[10] that of the pass that
 * fuses P6 and P7 where the iterations of `mode` run it in place of [5] and [6] (modes with no
 * SARA branch beside the data passes: PSARA_NNLS_INIT; 0 otherwise).  ms_per_pass holds
 * 11 doubles.  The iterations really run (the state advances by 2 * iters iterations). */
psara_status psara_profile_passes(psara_ctx* ctx, psara_mode mode, int iters, double* ms_per_pass);

/* Batched psara_solve_adaptive: every member stops on its own criteria (its launches then
 * do nothing for it) and the call returns when all have stopped or max_iters iterations have
 * run.  iters_run: NULL or `count` counts.  Each member's result equals its solo adaptive run. */
psara_status psara_batch_solve_adaptive(psara_ctx* const* ctxs, int count, psara_mode mode, int max_iters,
                                        int check_every, const psara_stop* stop, int* iters_run,
                                        psara_report* reports);

/* The same per-pass timing for a batch (the requirements of psara_batch_solve): every pass is
 * one launch over all `count` solves, all on the stream of ctxs[0] with the two branches
 * serialised, so each figure is the time of one batched launch of that pass.  ms_per_pass holds
 * 11 doubles.  Every member advances by 2 * iters iterations. */
psara_status psara_batch_profile_passes(psara_ctx* const* ctxs, int count, psara_mode mode, int iters,
                                        double* ms_per_pass);

/* ---- request server ---------------------------------------------------------------------- */

/* A server owns one GPU and solves submitted problems (Algorithm 2, each request with its own
 * operator, data and stage list) with continuous batching: requests are admitted while the sum
 * of their psara_footprint stays within the HBM budget (a request larger than the budget runs
 * when nothing else does; one larger than the device's whole memory is refused at submission
 * with PSARA_ENOMEM), set up by host threads while the GPU works, and every admitted request
 * advances in one batched launch per pass (grouped by stage mode, precision, tap count, image
 * side and check interval) in rounds of at most `quantum` iterations; a request leaves the
 * batch at each stage end for its reweighting and rejoins.  Policy PSARA_SERVE_FIFO instead runs
 * one request at a time in arrival order.  Each result equals the same request solved alone
 * with psara_* calls in the order the server uses (operator, data, prior with gamma 1, opnorm,
 * data gamma, psara_set_steps_auto with margin 0.99, the launch shapes stored for the request's
 * shape class if any (psara_tuning_lookup), then psara_reweighted_solve, or
 * psara_reweighted_solve_adaptive for a request with check_every > 0: such a request leaves the
 * batch as soon as its stage's criteria hold on the device).  Thread-safe for submit, poll and
 * cancel. */
typedef struct psara_server psara_server;

typedef enum { PSARA_SERVE_BATCHED = 0, PSARA_SERVE_FIFO = 1 } psara_serve_policy;

typedef struct {
  int n;                       /* image side (power of two, 8..1024) */
  int64_t M;                   /* visibility rows */
  const double* uv;            /* M x 2, rad/pixel in [-pi, pi)             (copied) */
  const double* Y;             /* M x 4 complex, interleaved, brightness order (copied) */
  double epsilon;              /* l2-ball radius, > 0 */
  int taps;                    /* 4, 6 or 8 */
  int levels;                  /* wavelet levels */
  uint32_t basis_mask;         /* bit 0 Dirac, bits 1..8 Db1..Db8 */
  psara_precision precision;
  psara_mode mode;             /* mode of the reweighted stages */
  int cycles;                  /* reweighting cycles; stages = cycles + 1 */
  const int* iters_per_stage;  /* cycles + 1 counts (copied) */
  double delta_decay;          /* > 1 */
  double gamma_factor;         /* gamma = gamma_factor ||Psi^dagger Re phi^dagger Y||_inf / ||phi||^2 */
  int opnorm_iters;            /* power-iteration limit and relative tolerance */
  double opnorm_rtol;
  int check_every;             /* 0: every stage runs its iters_per_stage iterations; > 0: a stage
                                  ends early when `stop` holds (psara_reweighted_solve_adaptive,
                                  tested every check_every iterations, iters_per_stage the bounds,
                                  each a multiple of check_every) */
  psara_stop stop;             /* stopping criteria when check_every > 0 */
} psara_request;

typedef enum { PSARA_REQ_QUEUED = 0, PSARA_REQ_RUNNING = 1, PSARA_REQ_DONE = 2, PSARA_REQ_FAILED = 3,
               PSARA_REQ_CANCELLED = 4 } psara_req_state;

typedef struct {
  int state;                   /* psara_req_state */
  psara_status status;         /* error of a failed request */
  double t_submit, t_start, t_done;   /* seconds on the server clock: submitted, set-up begun, result ready */
  int n;
  psara_report report;         /* final report of a finished request */
} psara_result;

/* device: GPU ordinal; hbm_budget: bytes of device memory the admitted requests may hold;
 * max_slots >= 1: most requests in flight; quantum >= 1: iterations per batched round. */
psara_status psara_server_create(psara_server** out, int device, size_t hbm_budget, int max_slots,
                                 int quantum, psara_serve_policy policy);
/* Queue a request (its arrays are copied before return); ticket receives its id.  PSARA_EINVAL
 * for a malformed request, PSARA_ENOMEM when its footprint exceeds the device's total memory
 * (it could never be admitted); the message is in psara_server_last_error. */
psara_status psara_server_submit(psara_server* srv, const psara_request* req, uint64_t* ticket);
/* Cancel a request: a queued one is removed at once, a running one at the worker's next step
 * (the end of the round in flight), which releases its device state, slot and footprint so
 * that queued requests can be admitted.  Its state becomes PSARA_REQ_CANCELLED (forgotten on
 * the first poll that reports it).  PSARA_EINVAL for an unknown ticket, PSARA_ESTATE when the
 * request has already ended. */
psara_status psara_server_cancel(psara_server* srv, uint64_t ticket);
/* State of a request.  When it is done and `image` is not NULL, the image (n*n x 4 doubles,
 * Stokes I, Q, U, V) is copied there and the request is forgotten (a later poll of the ticket
 * returns PSARA_EINVAL); a failed or cancelled request is forgotten on the first poll that
 * reports it. */
psara_status psara_server_poll(psara_server* srv, uint64_t ticket, psara_result* out, double* image);
/* Block until every submitted request has ended (done, failed or cancelled). */
psara_status psara_server_drain(psara_server* srv);
/* Seconds since the server was created (the clock of psara_result). */
double psara_server_clock(const psara_server* srv);
/* Message of the last failed request or call (valid until the next call of this function). */
const char* psara_server_last_error(const psara_server* srv);
/* Stops the threads after the running round and frees every context (pending requests are
 * dropped). */
void psara_server_destroy(psara_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* PSARA_H */
