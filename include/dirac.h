/*
 * dirac.h -- C ABI of libdirac, an MI355X (gfx950) implementation of the
 * directional-split pseudospectral time step ("Numerical Scheme II") for the
 * time-dependent Dirac equation in static curved 2-D space.
 *
 * Reference: X. Antoine, F. Fillion-Gourdeau, E. Lorin, S. McLean,
 * "Pseudospectral computational methods for the time-dependent Dirac equation
 * in static curved spaces", arXiv:1909.02894.
 *
 * One time step (Sec. 5.2, eqs. (poly_mod) and (second_scheme), 2-D form of
 * Numerical Experiment 3 with the absorbing layer of Sec. 3):
 *   1. psi <- E psi, E = exp(-i dt/2 [beta(x) m c^2 + F(x)])      (Step 1)
 *   2. x:  psi <- b_x F_1^{-1}[K_x(xi) F_1 psi] + (1 - b_x) psi     (direction 1)
 *   3. y:  psi <- b_y F_2^{-1}[K_y(xi) F_2 psi] + (1 - b_y) psi     (direction 2)
 *   4. psi <- E psi                                                 (Step 5)
 * with K_i(xi) = exp(-i c dt xi sigma_i), b_i = a(x)/S^i(x^i), a = e^{Phi-Psi}.
 *
 * Conventions shared by every call:
 *  - Every function returns dirac_status (0 = OK, < 0 = error); no C++
 *    exception crosses the ABI.  dirac_last_error() gives a thread-local
 *    message for the last failure on the calling thread.
 *  - A failed call leaves the solver as it was.
 *  - Host spinor arrays are complex128, layout [n2][n1][2] (y outer, x inner,
 *    spinor component innermost), each complex number as (re, im) doubles:
 *    4 doubles per grid point.  The caller owns them; they are copied.
 *  - The device buffer and the HIP stream are owned by the caller (for
 *    instance a torch uint8 tensor and torch's current stream); the library
 *    carves all of its device data out of that buffer and never frees it.
 *  - A solver handle is not thread safe.  Distinct handles on distinct
 *    streams may run concurrently.
 */
#ifndef DIRAC_H
#define DIRAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dirac_status;
enum {
    DIRAC_OK = 0,
    DIRAC_E_ARG = -1,        /* null pointer or out-of-range parameter          */
    DIRAC_E_SIZE = -2,       /* grid size not a power of two in [16, 8192], or a */
                             /* device buffer smaller than the footprint          */
    DIRAC_E_UNSTABLE = -3,   /* a blend coefficient b = a/S outside [0, 1]       */
    DIRAC_E_NOMEM = -4,      /* host allocation failed                          */
    DIRAC_E_DEVICE = -5,     /* a HIP call failed                               */
    DIRAC_E_STATE = -6,      /* call out of order (e.g. step before set_initial)*/
    DIRAC_E_NONFINITE = -7,  /* non-finite values in an input array              */
    DIRAC_E_NOCONV = -8      /* the Scheme I linear solve did not converge       */
};

/* Arithmetic of the state, FFTs and pointwise stages.  DIRAC_FP32 keeps the
 * tables generated in FP64 and rounded once, and all reductions in FP64. */
enum { DIRAC_FP64 = 0, DIRAC_FP32 = 1 };

/* Periodic grid on [-a1, a1) x [-a2, a2): x_i = -a1 + i h1, h1 = 2 a1 / n1
 * (Sec. 5).  n1, n2: powers of two in [16, 8192].  dt > 0, c > 0, m >= 0. */
typedef struct {
    int32_t n1, n2;
    double a1, a2;
    double dt, c, m;
} dirac_grid;

/* Static metric ds^2 = e^{2 Phi} dt^2 - e^{2 Psi} (dx^2 + dy^2) (Numerical
 * Experiment 3, Appendix A). */
enum {
    DIRAC_METRIC_FLAT = 0,        /* Phi = Psi = 0                                    */
    DIRAC_METRIC_GAUSS_BUMP = 1,  /* Phi = 0, Psi = ln(1 + |grad h|^2)/4,             */
                                  /* h = bump_A exp(-r^2 / bump_s^2) (static sheet)   */
    DIRAC_METRIC_PAPER_EXP3 = 2,  /* Phi = exp(-0.01 r^2), Psi = exp(-0.005 r^2)     */
    DIRAC_METRIC_FIELDS = 3       /* caller-given Phi, Psi and their gradients        */
};
/* Spin-connection potential chi: the Hamiltonian carries -i c a sigma_j d_j chi / 2. */
enum {
    DIRAC_SPIN_NONE = 0,   /* chi = 0                                               */
    DIRAC_SPIN_PAPER = 1,  /* chi = Phi (the printed 2-D equation)                   */
    DIRAC_SPIN_2P1 = 2     /* chi = Phi + Psi (conformal 2+1-D connection)          */
};
typedef struct {
    int32_t kind;                 /* DIRAC_METRIC_*                                  */
    int32_t spin;                 /* DIRAC_SPIN_*                                    */
    double bump_A, bump_s;        /* GAUSS_BUMP only (bump_s > 0)                    */
    /* FIELDS only: host arrays [n2][n1] of doubles, copied at create time. */
    const double *phi, *psi, *dphi_dx, *dphi_dy, *dpsi_dx, *dpsi_dy;
} dirac_metric;

/* Absorbing layer (Sec. 3): S^i = 1 + e^{i theta} Sigma~(x^i) on the width_pts
 * grid points next to the periodic seam x = +-a (layer L* <= |x| <= L, L = a,
 * L* = a - width_pts h; distance to the seam counted in whole grid steps).
 * type 1..6 = the paper's types I..VI with parameter sigma0.  width_pts = 0
 * switches the layer off.  Scheme II is stable only for real blend
 * coefficients in [0, 1] (stability proposition of Sec. 5.2), so a nonzero
 * theta inside an active layer is rejected with DIRAC_E_UNSTABLE. */
typedef struct {
    int32_t width_pts;
    int32_t type;
    double sigma0, theta;
} dirac_pml;

/* FP64 observables of the current state (dA = h1 h2):
 *   norm_l2 = dA sum |psi|^2,   norm_w = dA sum w |psi|^2 with w = e^{chi - Phi + Psi}
 *   (the weight the continuous equation conserves),
 *   energy = dA sum w psi^dag H psi with H the 2-D Hamiltonian of Numerical
 *   Experiment 3 (spectral derivative of eq. (trick), no layer stretch),
 *   x_mean, y_mean = density-weighted mean position, finite = 1 iff every
 *   state value is finite. */
typedef struct {
    int64_t step;
    double t;
    double norm_l2, norm_w, energy_re, energy_im, x_mean, y_mean;
    int32_t finite;
    int32_t reserved;
} dirac_obs;

typedef struct dirac_solver dirac_solver;

/* Time integrator.
 *  DIRAC_SCHEME_EXP_SPLIT (default): Numerical Scheme II, the exponential
 *    directional step of Sec. 5.2 (eq. (second_scheme)); needs real blend
 *    coefficients b = a/S in [0, 1].
 *  DIRAC_SCHEME_CN_GMRES: Numerical Scheme I of Sec. 5.1 (eq. (cn)): Step 1, the
 *    Crank-Nicolson transport step G psi* = G~ psi with
 *    G = I + (dt/2) alpha(x).T, G~ = I - (dt/2) alpha(x).T (spectral derivative of
 *    eq. (trick), alpha(x).T = c (b_x sigma_x d_x + b_y sigma_y d_y)), solved by
 *    restarted GMRES on the device, then Step 3.  Unconditionally stable for any
 *    real b (so b > 1 is accepted); FP64 only, n1, n2 <= 2048.
 *  DIRAC_SCHEME_EXP_SPLIT_2BIS_PRINTED: Scheme II with the directional step of
 *    eq. (step2bis) as printed, psi* = b Xi + (1-b) psi + b (c dt)^2 [[d^2]] Xi,
 *    i.e. the symbol K (1 - (c dt xi)^2).  First order in dt; |amplification| <= 1
 *    needs c dt max|xi| <= sqrt(2) on both axes (else DIRAC_E_UNSTABLE).
 *  DIRAC_SCHEME_EXP_SPLIT_2BIS: Scheme II with the second-order correction of the
 *    blend that eq. (step2bis) aims at: psi* = b Xi + (1-b) psi
 *    + ((c dt)^2/2) (-b(1-b) [[d^2]] psi + b b' [[d]] psi), b' = (d_i a)/S^i (the
 *    layer factor held fixed).  Second order in dt for the transport of each
 *    direction; explicit, so not unconditionally stable.  n1, n2 <= 2048. */
enum {
    DIRAC_SCHEME_EXP_SPLIT = 0,
    DIRAC_SCHEME_CN_GMRES = 1,
    DIRAC_SCHEME_EXP_SPLIT_2BIS_PRINTED = 2,
    DIRAC_SCHEME_EXP_SPLIT_2BIS = 3
};
typedef struct {
    int32_t scheme;          /* DIRAC_SCHEME_*                                         */
    int32_t gmres_restart;   /* Krylov vectors per cycle, 2..63 (0 = 20)                */
    int32_t gmres_max_iter;  /* total iterations per step before DIRAC_E_NOCONV (0 = 400) */
    int32_t reserved;        /* 0                                                      */
    double gmres_rtol;       /* stop at ||G x - b|| <= rtol ||b|| (0 = 1e-13)           */
} dirac_scheme;

/* Bytes of device memory a solver needs (including 256-byte alignment slack).
 * Returns 0 for invalid arguments. */
size_t dirac_footprint_bytes(const dirac_grid* grid, const dirac_metric* metric,
                             const dirac_pml* pml, int32_t precision);

/* Build a solver: validates the grid, builds every table on the device in FP64
 * (grid, momenta xi_p = p pi / a with the Nyquist index p = -n/2, metric fields,
 * a, the closed-form 2x2 half-step exponential E, layer profile 1/S, symbols
 * K_i, FFT twiddles, observable weights), checks the blend coefficients, and
 * synchronises the stream once.  device_buffer: caller-owned device memory of
 * at least dirac_footprint_bytes(...) bytes, 256-byte aligned.  hip_stream:
 * caller-owned hipStream_t (NULL = the null stream).  On success *out owns
 * host memory only; release it with dirac_destroy. */
dirac_status dirac_create_metric(const dirac_grid* grid, const dirac_metric* metric,
                                 const dirac_pml* pml, int32_t precision,
                                 void* device_buffer, size_t bytes, void* hip_stream,
                                 dirac_solver** out);

/* Time profile of a potential: f(t) = c0 + c1 sin(omega t + phase) g(t) with
 * g(t) = exp(-((t - t0) / tau)^2) for tau > 0, else g = 1. */
typedef struct {
    double c0, c1, omega, phase, t0, tau;
} dirac_envelope;

/* Electromagnetic potentials in F(t, x) (Sec. 2, the Hamiltonian with A and A0):
 * A0(t, x) = V(x) fV(t) and A_i(t, x) = A_i(x) fA(t).  In the conformal 2-D form
 * they add -e c a (A_x sigma_x + A_y sigma_y) - e A0 to beta m + F, so the Step 1 /
 * Step 5 exponential of step n is evaluated at t_{n+1/2} = (n + 1/2) dt
 * (eqs. (step1), (step3)), per point inside the direction kernels.  V, Ax, Ay are
 * host arrays [n2][n1] of doubles (NULL = 0), copied during creation; the step
 * index n counts from the last dirac_set_initial_spinor.  Schemes: the plain and
 * printed directional steps and Scheme I; n1, n2 <= 2048. */
typedef struct {
    const double* V;
    const double* Ax;
    const double* Ay;
    double charge;           /* e */
    dirac_envelope fV;       /* time profile of A0 */
    dirac_envelope fA;       /* time profile of (A_x, A_y) */
} dirac_em;

/* Footprint and creation with an explicit time integrator (scheme NULL = the
 * default Scheme II) and optional electromagnetic potentials (em NULL = none);
 * dirac_create_metric(...) = dirac_create_solver(..., NULL, NULL, ...) and
 * dirac_footprint_bytes_scheme(..., sc) = dirac_footprint_bytes_ex(..., sc, NULL). */
size_t dirac_footprint_bytes_scheme(const dirac_grid* grid, const dirac_metric* metric, const dirac_pml* pml,
                                    int32_t precision, const dirac_scheme* scheme);
size_t dirac_footprint_bytes_ex(const dirac_grid* grid, const dirac_metric* metric, const dirac_pml* pml,
                                int32_t precision, const dirac_scheme* scheme, const dirac_em* em);
dirac_status dirac_create_solver(const dirac_grid* grid, const dirac_metric* metric, const dirac_pml* pml,
                                 int32_t precision, const dirac_scheme* scheme, const dirac_em* em,
                                 void* device_buffer, size_t bytes, void* hip_stream, dirac_solver** out);

/* Scheme I statistics since creation: total GMRES iterations, and the relative
 * residual reached by the last solve. */
dirac_status dirac_cn_stats(const dirac_solver* s, int64_t* iterations, double* last_rel_residual);

/* Scheme I stopping rule of the solves that follow (Sec. 5.1: the linear system
 * of eq. (cn) is solved iteratively): at most max_iter >= 1 GMRES iterations per
 * step, stop at ||G x - b|| <= rtol ||b|| (rtol > 0).  A step that fails
 * (DIRAC_E_NOCONV, DIRAC_E_NONFINITE) leaves the state and step counter of the
 * whole dirac_step_n call as they were, so the call can be retried after
 * loosening the limits.  DIRAC_E_ARG for other schemes. */
dirac_status dirac_cn_set_limits(dirac_solver* s, int32_t max_iter, double rtol);

/* Upload the initial spinor psi^0 sampled at the grid points x_i = -a1 + i h1,
 * y_j = -a2 + j h2 of Sec. 5 (the collocation points of the partial DFTs
 * F_1, F_2 defined there): host [n2][n1][2] complex128, taken as given (not
 * normalised).  Resets the step counter and time to 0.  Synchronises the
 * stream.  DIRAC_E_NONFINITE if any value is not finite (nothing uploaded). */
dirac_status dirac_set_initial_spinor(dirac_solver* s, const double* psi_host);

/* Same from device memory: psi_dev holds [n2][n1][2] complex128 on the
 * solver's device (caller-owned, read before the next call on the stream
 * completes).  Asynchronous on the solver's stream; values are not checked. */
dirac_status dirac_set_initial_spinor_device(dirac_solver* s, const void* psi_dev);

/* Advance nsteps >= 0 time steps of the scheme chosen at creation.  Scheme II:
 * the Strang-split step of eq. (poly_mod) -- Step 1 (eq. (step1)), the x and y
 * directional steps of eq. (second_scheme) with the layer's a/S^i, Step 5
 * (eq. (step3)) -- asynchronously on the solver's stream.  Between consecutive
 * steps Step 5 and the next Step 1 are applied back to back in registers (E then
 * E), which is the same arithmetic as the unfused order.  Scheme I (eq. (cn)):
 * synchronous (the host drives the GMRES cycles); if a solve fails
 * (DIRAC_E_NOCONV, DIRAC_E_NONFINITE) the state and step counter are put back
 * to those at entry.  DIRAC_E_STATE before an initial spinor. */
dirac_status dirac_step_n(dirac_solver* s, int64_t nsteps);

/* Compute the observables of the current state into *out (caller-owned):
 * the discrete L2 norm of eq. (l2gamma) (dA sum over the grid), its weighted
 * form, and the energy with the spectral derivative of eq. (trick) (fields of
 * dirac_obs above).  Two derivative passes with fused FP64 partial sums, then
 * one fixed-order FP64 reduction: bitwise reproducible.  Synchronises the
 * stream.  DIRAC_E_STATE before an initial spinor. */
dirac_status dirac_observables(dirac_solver* s, dirac_obs* out);

/* Allocation-free observables, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same results as dirac_observables, bit for bit, but the
 * reduction partials and sums live in a static device array of the library
 * (1 MiB per GPU, held until the process ends; room for the 2 x 8192 workgroups
 * of the largest grid, DIRAC_E_SIZE beyond it) instead of the solver's buffer.
 * It calls no allocating routine.  Every call on one GPU shares that array:
 * calls that overlap on one GPU (solvers on different streams, or threads)
 * race and must be serialised by the caller.  Synchronises the solver's stream. */
dirac_status dirac_observables_static(dirac_solver* s, dirac_obs* out);

/* Copy the state psi^n at the grid points of Sec. 5 to host memory
 * (caller-owned, 4 n1 n2 doubles) as complex128 [n2][n1][2] (FP32 states are
 * widened exactly).  Synchronises. */
dirac_status dirac_get_spinor(dirac_solver* s, double* psi_host_out);

/* Release the handle (host memory only; the caller's device buffer is untouched). */
dirac_status dirac_destroy(dirac_solver* s);

/* Thread-local message for the last failed call on this thread ("" if none). */
const char* dirac_last_error(void);

/* --- schedules, timing and tuning ---------------------------------------------- */

/* FFT schedule of one direction: register radix (4, 8 or 16), lines (rows or
 * columns) per workgroup, and spinor components per thread (2: a thread holds
 * both components of its points; 1: the two components sit in partner lanes of
 * a wave).  Every per-line operation, and so every result bit, depends on
 * (n, precision, radix) only, never on lines_per_wg or components_per_thread. */
typedef struct {
    int32_t radix;
    int32_t lines_per_wg;
    int32_t components_per_thread;
} dirac_schedule;

/* Number of compiled schedules for (n, precision, direction 0 = x / 1 = y) and
 * the i-th of them. */
int32_t dirac_schedule_count(int32_t n, int32_t precision, int32_t direction);
dirac_status dirac_schedule_get(int32_t n, int32_t precision, int32_t direction, int32_t i,
                                dirac_schedule* out);

/* Read / override the schedules a solver uses (direction 0 = x, 1 = y). */
dirac_status dirac_get_schedule(const dirac_solver* s, int32_t direction, dirac_schedule* out);
dirac_status dirac_set_schedule(dirac_solver* s, int32_t direction, const dirac_schedule* sch);

/* State stores of the direction kernels, a bit mask: bit 0 for the x kernel,
 * bit 1 for the y kernel; a set bit selects device-scope write-through stores,
 * which send each line to memory at once instead of leaving it dirty in the
 * XCD's L2 until the kernel ends (0 = ordinary stores, the default).
 * Write-through pays on some small grids whose kernels are latency-bound and
 * loses on large streaming ones; dirac_autotune measures both per direction
 * and keeps the faster.  Results are bitwise the same either way.  Every form
 * of Scheme II's directional step (not Scheme I); write-through for the y
 * kernel only with n2 <= 1024 (else DIRAC_E_ARG). */
dirac_status dirac_set_store_mode(dirac_solver* s, int32_t write_through);
dirac_status dirac_get_store_mode(const dirac_solver* s, int32_t* write_through);

/* Launch mode of dirac_step_n: 0 = one kernel launch per stage, 1 = replay a
 * HIP graph of 2 * graph_chunk stage kernels (default, chunk 32). */
dirac_status dirac_set_launch_mode(dirac_solver* s, int32_t use_graph, int32_t graph_chunk);

/* Where a solve with potentials (Sec. 2, F(t, x)) evaluates the Step-1 / Step-5
 * exponentials E(t): form 1 = inside the direction kernels (one memory round
 * trip per direction), 2 = in a pointwise pass of their own before the x kernel
 * (and after the last y kernel) with the direction kernels in their plain
 * form, 0 = by size (default: the pass when the state and the potential record,
 * 12 reals a point, fit 128 MiB).  The two forms apply the same arithmetic in
 * the same order.  DIRAC_E_ARG for a solver without potentials or another
 * form.  dirac_get_potential_form reports 1 when the pass is in use, else 0. */
dirac_status dirac_set_potential_form(dirac_solver* s, int32_t form);
dirac_status dirac_get_potential_form(const dirac_solver* s, int32_t* pass);

/* Advance nsteps like dirac_step_n with one kernel launch per stage, each
 * launched with its own start/stop HIP events (hipExtLaunchKernel), so the
 * durations are the kernels' execution times in the x, y, x, y ... order of a
 * real run; then synchronise.  ms_out[0] / ms_out[1] = summed duration of the
 * x / y stage kernels in milliseconds, counts_out[0..1] = number of launches. */
dirac_status dirac_step_n_timed(dirac_solver* s, int64_t nsteps, double* ms_out,
                                int64_t* counts_out);

/* Average device time of one launch of each direction kernel: for each
 * direction, `reps` launches of that kernel alone (the mid-run form: the x
 * kernel applies Step 5 and Step 1, the y kernel neither) are recorded into a
 * HIP graph and replayed between two HIP events on the solver's stream.
 * us_out[0] / us_out[1] = microseconds per x / y launch (graph-internal
 * launch gaps included).  The state and the step counter are saved and
 * restored; synchronises.  Not for Scheme I or solves with time-dependent
 * potentials (DIRAC_E_ARG). */
dirac_status dirac_time_directions(dirac_solver* s, int32_t reps, double* us_out);

/* Autotuner: time every compiled schedule and store mode of each direction on
 * this solver's own buffers (the state is saved and restored, so the solve is
 * unchanged), x then y, twice over so each direction is tuned with the other's
 * choice in place; keep the fastest per (n, precision, direction, grid shape)
 * in a process-wide cache and apply it.  The corrected second-order step and
 * solves with potentials have one schedule per size: only their store modes
 * are searched.  Not for Scheme I (DIRAC_E_ARG).
 * reps = timed steps per candidate, in [1, 4096]; candidates run as in
 * dirac_step_n's graph mode. */
dirac_status dirac_autotune(dirac_solver* s, int32_t reps);

/* Save / load the tuning cache as a text file (one line per entry). */
dirac_status dirac_tune_cache_save(const char* path);
dirac_status dirac_tune_cache_load(const char* path);

/* --- batched solves ------------------------------------------------------------ */

/* A batch advances many independent solves of mixed grid sizes together: every
 * step of a run is two phases (direction x, then y); a phase covers all tiles
 * of all solves still running, with one kernel launch per transform length
 * present (each its own compiled schedule); lengths with too few tiles to fill
 * the GPU alone share one launch.  A run is recorded once into
 * a HIP graph and replayed.  Solves keep their own device buffers (created with
 * dirac_create_metric, same precision as the batch, n1 and n2 <= 2048); the
 * batch only holds descriptor tables in its own caller-given device buffer.
 * A solve's result depends on the radix of the schedules only, so it is
 * bitwise the same alone in a batch, in any mix, and in the single-solve path
 * with the same radix (dirac_set_schedule). */
typedef struct dirac_batch dirac_batch;

/* Device bytes for a batch of `capacity` solves. */
size_t dirac_batch_footprint_bytes(int32_t capacity);

dirac_status dirac_batch_create(int32_t precision, int32_t capacity, void* device_buffer, size_t bytes,
                                void* hip_stream, dirac_batch** out);

/* Put a solver (initial spinor already set) into a free slot; the batch then
 * launches its work on the batch stream.  *slot_out receives the slot index. */
dirac_status dirac_batch_add(dirac_batch* b, dirac_solver* s, int32_t* slot_out);

/* Take a solver out of its slot (the solver itself stays valid). */
dirac_status dirac_batch_remove(dirac_batch* b, int32_t slot);

/* Advance slot i by steps[i] >= 0 steps (steps has `capacity` entries; free
 * slots must have 0), asynchronously on the batch stream.  Each solve ends the
 * run on a step boundary, so observables and get_spinor work between runs
 * (after synchronising the batch stream, which dirac_batch_sync does). */
dirac_status dirac_batch_run(dirac_batch* b, const int64_t* steps);

/* Batch schedules: per direction and transform length n (a power of two in
 * [16, 2048]) the batch runs one of dirac_batch_schedule_count(n) schedules --
 * radix 8 or 4, one or both spinor components per thread, 256-thread
 * workgroups, lines per workgroup implied (lines_per_wg 0 = any).  Results
 * depend on the radix only.  dirac_batch_autotune times every valid schedule
 * for each (direction, n) present on `reps` steps of the whole batch, scored by
 * the summed duration of the kernels it can change (the size group's own kernel
 * and the kernel shared by the direction's small groups; per-launch events, the
 * best of three runs), keeps the lowest-numbered schedule within 1% of the
 * fastest, and restores every slot's state and step counter (synchronises). */
int32_t dirac_batch_schedule_count(int32_t n);
dirac_status dirac_batch_get_schedule(const dirac_batch* b, int32_t n, int32_t dir, dirac_schedule* out);
dirac_status dirac_batch_set_schedule(dirac_batch* b, int32_t n, int32_t dir, const dirac_schedule* sch);
dirac_status dirac_batch_autotune(dirac_batch* b, int32_t reps);

/* Prepare the run dirac_batch_run(b, steps) would launch -- upload its
 * descriptors and record and instantiate its HIP graph -- without launching
 * it or advancing any solve; the next dirac_batch_run with the same step
 * counts (and no slot change in between) only replays the graph.  No-op when
 * graphs are off.  Asynchronous on the batch stream. */
dirac_status dirac_batch_prepare(dirac_batch* b, const int64_t* steps);

/* dirac_batch_run with one kernel launch per size group and phase (no graph),
 * each launched with its own start/stop HIP events, then a synchronisation:
 * the durations are the kernels' execution times in the order of a real run.
 * Per kernel class c = direction * 9 + k (k = log2(n) - 4 for the kernel of the
 * size group of transform length n, k = 8 for the kernel shared by the small
 * groups): ms_out[c] = summed duration in milliseconds, counts_out[c] = number
 * of launches, bytes_out[c] = their algorithmic HBM bytes (each solve's state
 * read and written once per phase, plus its per-point tables: E and a in x, a
 * in y, for curved solves).  The three arrays have 18 caller-owned entries. */
dirac_status dirac_batch_run_timed(dirac_batch* b, const int64_t* steps, double* ms_out, int64_t* counts_out,
                                   double* bytes_out);

/* Wait for everything enqueued on the batch stream. */
dirac_status dirac_batch_sync(dirac_batch* b);

/* 0 = one launch per phase, 1 = record each run into a HIP graph (default). */
dirac_status dirac_batch_set_graph(dirac_batch* b, int32_t use_graph);

dirac_status dirac_batch_destroy(dirac_batch* b);

/* ------------------------------------------------------------------ 3-D ---
 * The 3-D, 4-spinor form of Scheme II (Sec. 5.2 with three directions): per
 * step, Step 1 (E), the x, y and z directional steps
 *   psi <- b_i F_i^{-1}[K_i F_i psi] + (1 - b_i) psi,
 *   K_i = exp(-i c dt xi alpha^i) = cos I - i sin alpha^i,  b_i = a / S^i,
 * and Step 5 (E), in the Dirac representation beta = diag(1, 1, -1, -1),
 * alpha^i = [[0, sigma_i], [sigma_i, 0]] (alpha^i = Pi^i Lambda Pi^{i,dag},
 * Lambda = diag(1, 1, -1, -1)).  E = exp(-i dt/2 [beta m c^2 e^Phi + F]) with
 * F = -i c a (alpha . grad chi) / 2 (the 2-D spin selectors carried over),
 * in closed form C I + D M since M^2 is a real multiple of I.
 * State: host [n3][n2][n1][4] complex128 (x fastest); device 8 T per point.
 * Sizes: powers of two in [16, 1024] per axis, state < 2 GiB.  Metrics:
 * DIRAC_METRIC_FLAT, DIRAC_METRIC_PAPER_EXP3 (Phi = exp(-0.01 r^2),
 * Psi = exp(-0.005 r^2), r^2 = x^2 + y^2 + z^2) and DIRAC_METRIC_FIELDS (eight
 * host planes [n3][n2][n1]).  The same real layer (dirac_pml) on every axis;
 * b = a / S in [0, 1] is required (DIRAC_E_UNSTABLE otherwise). */
typedef struct {
    int32_t n1, n2, n3;           /* points along x, y, z                         */
    double a1, a2, a3;            /* domain [-a1, a1) x [-a2, a2) x [-a3, a3)      */
    double dt, c, m;
} dirac3_grid;

typedef struct {
    int32_t kind;                 /* DIRAC_METRIC_FLAT, _PAPER_EXP3 or _FIELDS     */
    int32_t spin;                 /* DIRAC_SPIN_*                                  */
    const double *phi, *psi;      /* FIELDS only                                   */
    const double *dphi_dx, *dphi_dy, *dphi_dz, *dpsi_dx, *dpsi_dy, *dpsi_dz;
} dirac3_metric;

typedef struct {
    int64_t step;
    double t;
    double norm_l2;               /* h1 h2 h3 sum |psi|^2                          */
    double norm_w;                /* with the weight e^{chi - Phi + Psi}           */
    double x_mean, y_mean, z_mean;
    int32_t finite;
    int32_t reserved;
} dirac3_obs;

typedef struct dirac3_solver dirac3_solver;

size_t dirac3_footprint_bytes(const dirac3_grid* grid, const dirac3_metric* metric, const dirac_pml* pml,
                              int32_t precision);
dirac_status dirac3_create(const dirac3_grid* grid, const dirac3_metric* metric, const dirac_pml* pml,
                           int32_t precision, void* device_buffer, size_t bytes, void* hip_stream,
                           dirac3_solver** out);
dirac_status dirac3_set_initial_spinor(dirac3_solver* s, const double* psi_host);
dirac_status dirac3_set_initial_spinor_device(dirac3_solver* s, const void* psi_dev);
/* Asynchronous on the solver's stream (HIP-graph replay of 16-step chunks by default). */
dirac_status dirac3_step_n(dirac3_solver* s, int64_t nsteps);
dirac_status dirac3_set_launch_mode(dirac3_solver* s, int32_t use_graph, int32_t graph_chunk);
/* As dirac_step_n_timed, with ms_out[3] / counts_out[3] for the x, y, z kernels. */
dirac_status dirac3_step_n_timed(dirac3_solver* s, int64_t nsteps, double* ms_out, int64_t* counts_out);
dirac_status dirac3_observables(dirac3_solver* s, dirac3_obs* out);
dirac_status dirac3_get_spinor(dirac3_solver* s, double* psi_host_out);
dirac_status dirac3_destroy(dirac3_solver* s);

#ifdef __cplusplus
}
#endif
#endif /* DIRAC_H */
