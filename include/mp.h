/*
 * mp.h -- C ABI of the MI355X micropolar elastoplastic FFT-based solver.
 *
 * The library runs the elastoplastic FFT-based basic scheme of Francis,
 * Lebensohn, Pourahmadian and Dingreville (micropolar elastoplasticity with an
 * FFT-based solver): a Moulinec-Suquet fixed-point iteration on a periodic
 * voxel grid (Alg. 2) whose every iteration
 *   (a) forms the polarization stresses tau, mu (Eq. 34),
 *   (b) forward-transforms their 18 components,
 *   (c) applies the reference-medium Green operator per frequency (Eq. 35),
 *   (d) inverse-transforms to the strain and curvature fields and adds the
 *       prescribed averages E, Gamma,
 *   (e) runs the micropolar radial return (Alg. 1) at every voxel, and
 *   (f) evaluates the error measure of Eqs. 36-38.
 *
 * Conventions shared by every entry point
 *   - Grid n[0] x n[1] x n[2] voxels of size h, x fastest: voxel (x, y, z) has
 *     linear index (z * n[1] + y) * n[0] + x.  Every n[i] must be one of
 *     4 6 8 12 16 24 32 48 64 96 128 192 256.
 *   - Tensor V_kl is component 3 * k + l (k = row).  t_kl acts on the face of
 *     normal k (Eq. 2); e_kl = u_l,k + eps_lkm phi_m, gamma_kl = phi_k,l (Eq. 1);
 *     m_kl = B_lkmn gamma_mn (Eq. 5).
 *   - Device fields are structure-of-arrays: component c of a 9-component
 *     field occupies n voxels starting at c * n.
 *   - Frequencies are the continuous ones, xi = 2 pi m / (n h).  The
 *     fluctuating strain and curvature are zero at k = 0 and at every Nyquist
 *     index.
 *   - All work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL = default stream).  Device memory comes from the caller: the
 *     library allocates none (its one static device buffer, that of
 *     mp_green_apply_noalloc, aside).  Host arrays are copied during the call
 *     and never retained.
 *   - Errors are returned as mp_status; mp_last_error() gives a thread-local
 *     message.  No C++ exception crosses this boundary.
 */
#ifndef MP_H
#define MP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MP_OK = 0,
  MP_E_INVALID = 1,        /* bad argument or unsupported problem */
  MP_E_NOMEM = 2,          /* workspace smaller than mp_plan_workspace_size */
  MP_E_DEVICE = 3,         /* a HIP call failed */
  MP_E_NOT_CONVERGED = 4,  /* max_iter reached in a step; that step is committed */
  MP_E_DIVERGED = 5,       /* non-finite error measure, or one grown 1e6 x above the
                              step's smallest; that step is not committed and the
                              plan (or batched RVE) takes no further steps */
  MP_E_STATE = 6           /* call not valid in the plan's current state */
} mp_status;

enum { MP_FP64 = 0, MP_MIXED = 1 };                 /* arithmetic of the bulk fields */
enum { MP_ERR_LOCAL = 0, MP_ERR_AVERAGE = 1 };      /* Eq. 38 | Eq. 37 */
/* Reference medium A0, B0 (Alg. 2).  PHASE_MEAN, VOLUME_MEAN and EXPLICIT
 * give an isotropic medium (Eq. 6 constants: the unweighted mean over the
 * phases present, the volume average, or mp_problem.ref), whose Green
 * operator (Eqs. 33-35) has a closed form.  TENSOR_MEAN takes Alg. 2
 * literally with every phase's own tensors: A0 = <A(x)>, B0 = <B(x)> over
 * the cell, Eq. 5 tensors where a phase has them (mp_aniso), Eq. 6 ones
 * elsewhere; TENSOR_PHASE_MEAN is the unweighted mean of those tensors over
 * the phases present (like PHASE_MEAN, it keeps the basic scheme convergent
 * when a stiff phase fills a small volume).  With a tensor reference the
 * Green operator factors the 6x6 Fourier symbol at every frequency (it is
 * positive definite whenever <A> is, which valid phases ensure; <B> may be
 * singular on skew tensors, gamma = beta). */
enum { MP_REF_PHASE_MEAN = 0, MP_REF_VOLUME_MEAN = 1, MP_REF_EXPLICIT = 2, MP_REF_TENSOR_MEAN = 3,
       MP_REF_TENSOR_PHASE_MEAN = 4, MP_REF_GEOMETRIC_MEAN = 5 };
/* MP_REF_GEOMETRIC_MEAN: the unweighted geometric mean of each Eq. 6 modulus
 * over the phases present (0 where a phase has a zero modulus), the penalty
 * Michel, Moulinec and Suquet give for the augmented-Lagrangian scheme. */
/* Fixed-point scheme of every load step.  BASIC: Alg. 2's loop.  AL: the
 * augmented-Lagrangian scheme the paper's conclusion names for high phase
 * contrast, in its alternating-direction form with the reference medium as
 * the penalty C0.  Each iteration forms the compatible field e = E + G0
 * (s(d) - C0 d) from the local strain d (the Green operator of Eqs. 33-35 on
 * the polarization of Eq. 34 at d), over-relaxes it, e^ = w e + (1 - w) d,
 * and solves the local step s(d') + C0 d' = s(d) + C0 e^ voxel by voxel, s
 * the stress of Alg. 1 (the multiplier equals s(d) after every step and is
 * not stored).  Its fixed point is Alg. 2's; the error measure (Eqs. 36-38)
 * is taken on d and s(d), with the prescribed E, Gamma in the strain
 * denominators.  AL needs MP_FP64, phases without Eq. 5 tensors, an
 * isotropic reference medium with gamma0 > beta0 unless every phase present
 * has gamma = beta, and 0 < relax < 2; it runs in plans and in FP64 batches
 * (beside basic-scheme RVEs of the same shape). */
enum { MP_SCHEME_BASIC = 0, MP_SCHEME_AL = 1 };
/* How the Green operator of the reference medium (Eqs. 33-35) is evaluated.
 * COMPUTED: at every frequency of every iteration, in closed form for an
 * isotropic medium or by factoring its 6x6 Fourier symbol for a tensor one.
 * STORED: as the paper precomputes it (Sec. 2.4): mp_plan_create writes the
 * 21 entries of the inverse symbol at every frequency of the half spectrum
 * into the workspace (21 n0/2 n1 n2 words of the bulk precision; FP64
 * entries rounded to FP32 under MP_MIXED), and each iteration reads them.
 * The two give the same operator up to rounding.  Plans and batches (a
 * batch builds an RVE's table when it admits it; mp_batch_footprint counts
 * it). */
enum { MP_GREEN_COMPUTED = 0, MP_GREEN_STORED = 1 };
enum { MP_FIELD_E = 0, MP_FIELD_GAMMA = 1, MP_FIELD_T = 2, MP_FIELD_M = 3,
       MP_FIELD_P = 4, MP_FIELD_Q = 5 };

/* Constants of one isotropic phase: Eq. 6 moduli, Eqs. 13-18 plastic
 * constants.  tY = +inf (resp. mY = +inf) makes the macro (micro) level
 * purely elastic.  Alg. 1 derives a2 = a1 mu / kappa and
 * b2 = b1 (gamma + beta) / (gamma - beta); gamma == beta is accepted and
 * means a vanishing skew couple-stress modulus (the b2 term then drops). */
typedef struct {
  double lambda, mu, kappa, alpha, beta, gamma;
  double tY, tH, mY, mH, a1, b1;
} mp_phase;

/* A phase with general centrosymmetric elastic tensors (Eq. 5) in place of
 * the isotropic ones of Eq. 6.  Both tensors must be symmetric over their
 * index pairs (A_klmn = A_mnkl, B_lkmn = B_mnlk) and positive definite as
 * 9 x 9 matrices.  The phase must be elastic (tY = mY = INFINITY); its
 * tensors enter an MP_REF_TENSOR_* reference medium, and its isotropic
 * constants in mp_phase the isotropic reference media and the Eqs. 14, 17
 * equivalent stresses reported as Teq, Meq. */
typedef struct {
  int32_t phase;            /* phase id (< n_phases), listed at most once */
  double A[81];             /* A_klmn at index 27k + 9l + 3m + n: t_kl = A_klmn e_mn */
  double B[81];             /* B_lkmn at index 27l + 9k + 3m + n: m_kl = B_lkmn gamma_mn */
} mp_aniso;

/* Problem statement (inputs of Alg. 2). */
typedef struct {
  int32_t n[3];             /* voxels along x, y, z */
  double h;                 /* voxel size */
  const uint8_t* phase;     /* host, n[0]*n[1]*n[2] phase ids, each < n_phases */
  int32_t n_phases;         /* 1..256 */
  const mp_phase* phases;   /* host, n_phases records */
  int32_t ref_mode;         /* MP_REF_*: reference medium A0, B0 */
  mp_phase ref;             /* elastic constants used with MP_REF_EXPLICIT */
  double tol;               /* epsilon of Alg. 2 (> 0) */
  int32_t max_iter;         /* loop cap per step (>= 1) */
  int32_t err_norm;         /* MP_ERR_LOCAL | MP_ERR_AVERAGE */
  int32_t precision;        /* MP_FP64, or MP_MIXED: the spectra, the history
                               base and the committed stresses are stored in
                               FP32 and the transforms and the Green operator
                               run in FP32; the strain state, the return map
                               (Alg. 1), the polarization, p, q, the error
                               measure (Eqs. 36-38) and every volume average
                               stay FP64.  After a step's first iteration the
                               transforms carry the polarization's increment
                               (the Green operator is linear), so their
                               rounding shrinks with it and every step ends at
                               tol like FP64 */
  int32_t n_aniso;          /* phases with Eq. 5 tensors, 0..n_phases */
  const mp_aniso* aniso;    /* host, n_aniso records (unused when n_aniso = 0) */
  int32_t scheme;           /* MP_SCHEME_BASIC (0) | MP_SCHEME_AL */
  double relax;             /* MP_SCHEME_AL: over-relaxation w, 0 < w < 2 (1: none) */
  int32_t green_mode;       /* MP_GREEN_COMPUTED (0) | MP_GREEN_STORED */
} mp_problem;

typedef struct mp_plan_s* mp_plan;

/* Bytes of device workspace a plan for `prob` needs.  Validates `prob`
 * (Eq. 7 bounds with gamma - beta >= 0 allowed, kappa > 0, alpha = 0 in any
 * phase with finite mY, tY > 0, mY > 0, grid sizes) and returns
 * MP_E_INVALID on violation. */
mp_status mp_plan_workspace_size(const mp_problem* prob, size_t* bytes);

/* Create a plan: carves `dev_workspace` (>= mp_plan_workspace_size bytes,
 * 256-byte aligned, owned by the caller, must outlive the plan), uploads the
 * phase map and constants, computes the reference medium (Alg. 2: A0 from
 * the phases; default the unweighted mean of each modulus over the phases
 * present) and sets the zero initial state of Alg. 2.  Work goes to
 * `hip_stream`. */
mp_status mp_plan_create(const mp_problem* prob, void* dev_workspace, size_t bytes,
                         void* hip_stream, mp_plan* out);

/* Solve load steps with Alg. 2, continuing from the plan's current state.
 * times: n_steps + 1 values; times[0] is the time of the current state (the
 * zero state for a fresh plan), times[s] the end of step s.  E, Gam:
 * [n_steps][9] prescribed average strain and curvature at times[1..].
 * iters: optional [n_steps] output of loop iterations per step.
 * The first step of a fresh plan starts from the uniform E; later steps start
 * from the linear extrapolation of the last two committed states.  Returns
 * at the first step that does not converge: MP_E_NOT_CONVERGED after
 * committing it, MP_E_DIVERGED without committing it (the plan then returns
 * MP_E_STATE to later calls).  Blocks until the work is done. */
mp_status mp_solve_load_path(mp_plan plan, int32_t n_steps, const double* times,
                             const double* E, const double* Gam, int32_t* iters);

/* Homogenized response of committed step `step` (1-based, counted over the
 * plan's life).  out[42] = T[9] M[9] <e>[9] <gamma>[9] <p> <q> <t_eq> <m_eq>
 * err iterations, all volume averages in FP64. */
mp_status mp_homogenized_response(mp_plan plan, int32_t step, double out[42]);

/* The four terms of the error measure (Eq. 36) at the end of committed step
 * `step`: out[5] = err_e, err_t, err_gamma, err_m (Eq. 38 or Eq. 37), and a
 * reserved 0.0. */
mp_status mp_step_error_parts(mp_plan plan, int32_t step, double out[5]);

/* Copy fields of the state after the last committed step as FP64 values (the
 * outputs of Alg. 2): bit f of `mask` (1 << MP_FIELD_*) selects field f,
 * written to dst[f] (dst holds 6 pointers indexed by field id; unselected
 * entries are not read).  MP_FIELD_E/GAMMA/T/M receive 9*n doubles (SoA,
 * component 3k + l), MP_FIELD_P/Q n doubles.  dst_is_device = 0: host
 * destinations, the call returns when they are written; 1: device
 * destinations, the copies (FP32 stresses of MP_MIXED widened on the device)
 * are enqueued on the plan's stream and the call returns without waiting.
 * e and gamma are the last iterate, the committed one unless a step diverged
 * (MP_E_DIVERGED leaves its iterate there and the stresses of the last
 * committed step).  MP_E_INVALID for mask bits beyond MP_FIELD_Q or a NULL
 * selected destination. */
mp_status mp_get_fields(mp_plan plan, uint32_t mask, void* const* dst, int32_t dst_is_device);

/* Test hook: when n_fixed > 0 every later step runs exactly n_fixed loop
 * iterations regardless of the tolerance (0 restores the tolerance test).
 * Lets parity tests follow a given iteration schedule. */
mp_status mp_set_fixed_iterations(mp_plan plan, int32_t n_fixed);

/* Eigenstress: the verification form of the polarization used by the
 * method of numerically manufactured solutions (App. D.1, the manufactured
 * polarization equation), tau = t - A0 e - tau_m, mu = m - B0 gamma - mu_m.
 * dev_eig: 18*n device values of the plan's precision (double for MP_FP64,
 * float for MP_MIXED), SoA [c][voxel] with c = 3k + l for tau_m (0..8) and
 * 9 + 3k + l for mu_m.  The caller owns the buffer; it is read, not copied,
 * by every polarization of later mp_solve_load_path calls until it is
 * replaced, or cleared with NULL.  A manufactured stress that changes from
 * step to step is set before each single-step call. */
mp_status mp_set_eigenstress(mp_plan plan, const void* dev_eig);

/* Number of committed steps. */
mp_status mp_plan_steps(mp_plan plan, int32_t* steps);

/* Apply the spectral part of one iteration (rows b-d above) to given
 * polarization fields: in = 18*n device doubles (tau then mu, SoA), out =
 * 18*n device doubles receiving the fluctuating strain then curvature
 * (no averages added).  Uses the plan's transforms and reference medium. */
mp_status mp_green_apply(mp_plan plan, const void* dev_in, void* dev_out);
/* (mp_green_apply, mp_spectrum_forward and mp_radial_return accept FP64
 * plans only and return MP_E_INVALID for MP_MIXED plans.) */

/* Allocation-free variant of mp_green_apply, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Applies rows b-d above to 18 real FP64
 * fields without a plan: forward transform, the Green operator of the
 * isotropic reference medium ref = {lambda0, mu0, kappa0, alpha0, beta0,
 * gamma0} (Eq. 6 constants) on the grid n[0] x n[1] x n[2] of voxel size h,
 * inverse transform.  dev_in: 18*n device doubles (tau then mu, SoA,
 * component 3k + l); dev_out: 18*n device doubles receiving the fluctuating
 * strain then curvature (no averages added); they must not overlap; both
 * stay owned by the caller.  The half spectra and the twiddle tables live in
 * a static device buffer of the library, 48 MiB on every device it runs on,
 * held until the process ends: 18 * n[2] * n[1] * (n[0]/2) * 16 bytes plus
 * the twiddles must fit (every grid up to 64^3 does); a larger grid, an
 * unsupported size, h <= 0 or a reference that is not positive definite
 * gives MP_E_INVALID before any device work.  The call allocates nothing and
 * does not synchronise: the work is enqueued on hip_stream and the buffer is
 * in use until it has run.  Every call on one device shares that device's
 * buffer, which keeps the last call's contents: calls that overlap in time on
 * one device (different streams or threads) race and corrupt each other's
 * results; calls ordered on one stream are safe.  The results equal
 * mp_green_apply's on an FP64 plan with the same grid, h and reference
 * medium, up to the rounding of the twiddles (computed on the device here). */
mp_status mp_green_apply_noalloc(const int32_t n[3], double h, const double ref[6],
                                 const void* dev_in, void* dev_out, void* hip_stream);

/* Forward transform of 18 real fields (device, 18*n doubles, SoA) to their
 * half spectra: dev_out receives n[2] * n[1] * (n[0]/2) * 18 complex doubles
 * (interleaved re, im), component-interleaved layout [kz][ky][kx][c],
 * kx = 0 .. n[0]/2 - 1 (the x-Nyquist bin is not kept), unnormalised
 * forward DFT.  This is the solver's own spectral layout. */
mp_status mp_spectrum_forward(mp_plan plan, const void* dev_in, void* dev_out);

/* Radial return (Alg. 1) at n_vox independent points on the device, FP64.
 * phase: n_vox uint8 ids into the plan's phase table.  e, g, e_n, g_n, t_n,
 * m_n: 9*n_vox SoA; p_n, q_n: n_vox.  Outputs t, m (9*n_vox), p, q (n_vox).
 * Uses the same device code as the solver (trial stresses formed from the
 * history base t_n - A e_n, m_n - B g_n).  MP_E_INVALID for a plan whose
 * problem has Eq. 5 phases (n_aniso > 0). */
mp_status mp_radial_return(mp_plan plan, int64_t n_vox, const void* phase,
                           const void* e, const void* g, const void* e_n, const void* g_n,
                           const void* t_n, const void* m_n, const void* p_n, const void* q_n,
                           void* t, void* m, void* p, void* q);

/* Per-kernel timing of loop iterations, for measurement.  mode 1: the plan
 * records hipEvents on its stream between the kernels of every iteration
 * that runs and accumulates their durations; mode 2: events around the x
 * pass only (two records per iteration, the least added to the loop);
 * mode 0: off.  Counters reset on every call.  mp_profile_read fills
 * ms_total[j] (milliseconds) and launches[j] for j < min(n, 5), kernel j in
 * iteration order: 0 y forward, 1 z forward + Green operator + z inverse,
 * 2 y inverse, 3 x pass (inverse x transform, return maps, error partials,
 * polarization, forward x transform), 4 error reduction.  Each event record
 * adds a few microseconds between two kernels.  A plan of a small cell
 * (FP64, every axis 4 or 8 long, isotropic computed Green operator, basic
 * scheme) otherwise runs a step's loop in one kernel; with timing on it
 * runs these kernels apart, with bit-for-bit equal iterates. */
mp_status mp_profile(mp_plan plan, int32_t mode);
mp_status mp_profile_read(mp_plan plan, int32_t n, double* ms_total, int64_t* launches);

void mp_plan_destroy(mp_plan plan);
const char* mp_last_error(void);
const char* mp_version(void);

/* ------------------------------------------------------------------------
 * Resident batches: many independent RVEs, of a few shape classes, solved
 * together.  Each admitted RVE keeps its whole state in the batch's device
 * arena and runs its own load path with Alg. 2 (own convergence, step
 * control, extrapolation and commit) entirely on the device.  One
 * mp_batch_run replays a captured graph of iters_per_launch loop iterations
 * of every resident RVE (per shape class: y forward, z forward + Green
 * operator + z inverse, y inverse, x pass; then one reduction and one
 * control kernel for the whole batch).  An RVE solved in a batch goes
 * through the same arithmetic, in the same order, as with mp_plan, so its
 * results are identical to a solo solve of the same problem.
 * ------------------------------------------------------------------------ */
typedef struct mp_batch_s* mp_batch;

typedef struct {
  int32_t precision;         /* MP_FP64 | MP_MIXED, for every RVE of the batch */
  int32_t n_shapes;          /* number of shape classes, 1..8 */
  int32_t shapes[8][3];      /* n[0], n[1], n[2] of each class */
  int32_t max_rves;          /* resident RVEs at most, 1..512 */
  int32_t iters_per_launch;  /* loop iterations per graph launch, 1..64 */
  int32_t autotune;          /* 1: at creation, time each class's y / z tile
                                widths {1, wide/2, wide} with the full
                                persistent grid, a quarter of it and the
                                blocks the chip holds at once, and keep the
                                fastest (cached per shape for the process);
                                0: the single-plan tile widths */
} mp_batch_config;

enum { MP_RVE_RUNNING = 0, MP_RVE_DONE = 1 };

/* Arena bytes one RVE of `prob` with n_steps load steps takes in a batch of
 * configuration `cfg` (fields, spectra, history, phase map, constants, load
 * path, step records).  Admission succeeds while this fits in the arena. */
mp_status mp_batch_footprint(const mp_batch_config* cfg, const mp_problem* prob, int32_t n_steps,
                             size_t* bytes);

/* Create an empty batch on the caller's device arena (256-byte aligned,
 * owned by the caller, must outlive the batch; about 0.6 MB of it holds the
 * slot descriptors).  Work goes to `hip_stream`.  Tunes the schedules when
 * cfg->autotune is set. */
mp_status mp_batch_create(const mp_batch_config* cfg, void* dev_workspace, size_t bytes,
                          void* hip_stream, mp_batch* out);

/* Admit one RVE: validate (as mp_plan_workspace_size), place it in the arena
 * and a free slot, upload its phase map, constants and load path (times:
 * n_steps + 1 values from the zero state; E, Gam: [n_steps][9]).  It starts
 * at the next mp_batch_run.  prob->precision must equal the batch's; the
 * grid must be one of its shape classes.  MP_E_NOMEM when the arena or the
 * slots are full (nothing changes).  *id identifies it until released. */
mp_status mp_batch_admit(mp_batch batch, const mp_problem* prob, int32_t n_steps, const double* times,
                         const double* E, const double* Gam, int32_t* id);

/* One graph launch: iters_per_launch loop iterations (step transitions
 * included) of every resident, unfinished RVE.  *n_active receives the
 * number still unfinished.  Blocks. */
mp_status mp_batch_run(mp_batch batch, int32_t* n_active);

/* Graph launches as mp_batch_run until no RVE is unfinished (or
 * max_launches > 0 launches).  From the second launch on, each launch is
 * queued before the state after the previous one is read back, so the host's
 * checks overlap the GPU's work; the one launch queued after the last RVE
 * finished finds no work and changes nothing.  *launches counts every
 * launch.  Blocks. */
mp_status mp_batch_drain(mp_batch batch, int32_t max_launches, int32_t* launches);

/* State (MP_RVE_RUNNING | MP_RVE_DONE), status (MP_OK, MP_E_NOT_CONVERGED or
 * MP_E_DIVERGED, as mp_solve_load_path would return it), committed steps and
 * loop iterations so far of RVE `id`. */
mp_status mp_batch_query(mp_batch batch, int32_t id, int32_t* state, int32_t* status,
                         int32_t* steps_done, int64_t* iters_total);

/* Record of committed step `step` (1-based) of RVE `id`: out[0..41] as
 * mp_homogenized_response, out[42..46] as mp_step_error_parts, out[47] 0. */
mp_status mp_batch_response(mp_batch batch, int32_t id, int32_t step, double out[48]);

/* Fields of RVE `id` (after its last committed step), as mp_get_fields (device
 * copies go to the batch's stream). */
mp_status mp_batch_get_fields(mp_batch batch, int32_t id, uint32_t mask, void* const* dst,
                              int32_t dst_is_device);

/* Test hook, as mp_set_fixed_iterations for RVE `id`: with n_fixed > 0
 * every step of it runs exactly n_fixed loop iterations (0 restores the
 * tolerance test); applies from its current step on.  Call between launches. */
mp_status mp_batch_set_fixed_iterations(mp_batch batch, int32_t id, int32_t n_fixed);

/* Remove RVE `id` (cancelling it if unfinished) and return its arena region. */
mp_status mp_batch_release(mp_batch batch, int32_t id);

/* Schedule of shape class `cls`: out = {y-forward TX, grid, z TX, grid,
 * y-inverse TX, grid, x-pass grid, x tiles per RVE}; ms (optional, 3 values)
 * the autotuner's per-RVE time of each y / z pass (0 when not tuned). */
mp_status mp_batch_schedule(mp_batch batch, int32_t cls, int32_t out[8], float ms[3]);

/* Graph launches so far, arena bytes in use, resident RVEs. */
mp_status mp_batch_stats(mp_batch batch, int64_t* graph_launches, size_t* arena_used,
                         int32_t* resident);

void mp_batch_destroy(mp_batch batch);

/* ------------------------------------------------------------------------
 * Serving: requests (an RVE and its load path) arrive over time; the reply
 * is the solved path.  Times are seconds from the start of the call, taken
 * from a steady clock while the requests are served in real time.
 * ------------------------------------------------------------------------ */
typedef struct {
  double arrival;            /* seconds after the start, non-decreasing */
  const mp_problem* prob;
  int32_t n_steps;
  const double* times;       /* n_steps + 1 */
  const double* E;           /* [n_steps][9] */
  const double* Gam;         /* [n_steps][9] */
  /* the reply, written before the request counts as done (caller-owned): */
  double* records;           /* [n_steps][48] host doubles, the step records as
                                mp_batch_response gives them; rows of steps not
                                committed (the request failed) are NaN; NULL: none */
  uint32_t field_mask;       /* fields of the final state (1 << MP_FIELD_*), 0: none */
  void* fields[6];           /* their destinations by field id, as mp_get_fields */
  int32_t fields_on_device;  /* 1: fields[] are device pointers (the copies are
                                complete when the request is done) */
} mp_request;

/* Continuous batching on an empty batch: arrived requests are admitted in
 * arrival order while their footprint fits in the free arena (a later
 * request may pass a head that does not fit, until the head has been passed
 * max_bypass times); resident RVEs keep their state across launches;
 * finished ones are retired after every graph launch: their replies (step
 * records, fields) are read back, then their region is freed for the queue.
 * Requests are solved in the batch's precision.  Per request: t_admit,
 * t_done (seconds, after the reply is written), status, loop iterations.  With
 * progress_s > 0 a progress line goes to stderr every progress_s seconds. */
mp_status mp_serve_batched(mp_batch batch, int32_t n, const mp_request* req, int32_t max_bypass,
                           double progress_s, double* t_admit, double* t_done, int32_t* status,
                           int64_t* iters);

/* The same requests served one at a time in arrival order with FP64 plans
 * (mp_plan_create / mp_solve_load_path / mp_plan_destroy) on a workspace of
 * `bytes`, each reply written as above.  Per request: t_start, t_done
 * (seconds, after the reply), status, iterations.
 * With progress_s > 0 a line goes to stderr after every request (and
 * while waiting, at least every progress_s seconds the call returns to its
 * clock). */
mp_status mp_serve_sequential(int32_t n, const mp_request* req, void* dev_workspace, size_t bytes,
                              void* hip_stream, double progress_s, double* t_start, double* t_done,
                              int32_t* status, int64_t* iters);

#ifdef __cplusplus
}
#endif
#endif /* MP_H */
