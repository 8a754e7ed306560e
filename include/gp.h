/*
 * gp.h -- C ABI of libgp: split-step Crank-Nicolson (SSCN) time steps of the
 * dimensionless Gross-Pitaevskii equation on one AMD Instinct MI355X (gfx950).
 *
 *     i dpsi/dt = [ -1/2 laplacian + V + g |psi|^2 ] psi,   V = 1/2 sum_a w_a^2 x_a^2
 *
 * The paper's program summary ("Nature of problem", "Solution method") defines
 * the problem -- 1d/2d/3d condensates in fully anisotropic harmonic traps --
 * and the method: split-step Crank-Nicolson discretisation in space and time,
 * propagated in imaginary time (stationary states) or real time (dynamics);
 * "Summary of revisions" lists the outputs (energy, chemical potential, rms
 * sizes).  One step, as computed here:
 *   1. pointwise potential + nonlinear propagator, |psi|^2 taken before it:
 *        real time  psi <- psi exp(-i theta),  imaginary time psi <- psi exp(-theta),
 *        theta = dt (V + g |psi|^2);
 *   2. one Crank-Nicolson kinetic substep per axis, x then y then z, each a
 *      constant-coefficient tridiagonal solve along every grid line
 *      (3-point Laplacian, zero values at the ghost points i = -1 and i = N_a);
 *   3. imaginary time only: renormalise to dV sum |psi|^2 = 1.
 * Grid: x_{a,i} = (i - N_a/2) dx_a, i = 0..N_a-1;  dV = prod dx_a.
 *
 * Conventions shared by every entry point
 *  - Wavefunctions are caller-owned DEVICE buffers of interleaved (re, im)
 *    values, complex128 (GP_C128) or complex64 (GP_C64), dense, x fastest:
 *    element (i, j, k) at i + N0 (j + N1 k).  A torch tensor of shape
 *    (Nz, Ny, Nx) and dtype complex128/complex64 has exactly this layout.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it; only gp_observables, gp_plan_timing_read and the
 *    batch autotuner synchronise it.
 *  - Every function returns gp_status and never throws or aborts.  Arguments
 *    are checked before any HIP call.  An asynchronous device fault surfaces as
 *    GP_EHIP on a later call.  gp_last_error() gives a message for the last
 *    failure on the calling thread.
 *  - A plan is not thread-safe; separate plans may run on separate streams.
 *    A plan binds to the device that is current when it is created.
 */
#ifndef GP_H
#define GP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GP_OK = 0,
    GP_EINVAL = -1,        /* bad argument (null pointer, size, dt, dx, enum) */
    GP_ENOMEM = -2,        /* device or host allocation failed */
    GP_EHIP = -3,          /* HIP runtime error (message in gp_last_error) */
    GP_ENONFINITE = -4,    /* non-finite norm or energy found */
    GP_EUNSUPPORTED = -5,  /* valid request this build does not implement */
    GP_ETIMEOUT = -6       /* a bounded device-side wait gave up */
} gp_status;

typedef enum { GP_IMAG = 0, GP_REAL = 1 } gp_mode;

/* GP_C64: complex64 storage and FP32 arithmetic for the bulk of the step, with
 * FP64 norm/energy reductions and an FP64 renormalisation factor. */
typedef enum { GP_C128 = 0, GP_C64 = 1 } gp_prec;

/* Harmonic trap V = 1/2 sum_a omega[a]^2 x_a^2.  Optionally a host array of
 * per-step frequencies replaces omega[sched_axis] in the potential substep of
 * step n for 0 <= n < sched_len (the plan copies it); later steps use the
 * static omega[].  Observables use the trap of the plan's last step. */
typedef struct {
    double omega[3];
    const double *omega_sched;
    int64_t sched_len;
    int sched_axis;
} gp_trap;

/* Observables (rectangle sums over the grid, FP64 accumulation):
 *   norm  = dV sum |psi|^2
 *   ekin  = dV/2 sum_a sum_lines sum_{i=-1}^{N_a-1} |u_{i+1}-u_i|^2 / dx_a^2  (zero ghosts)
 *   epot  = dV sum V |psi|^2,   eint = g dV/2 sum |psi|^4
 *   energy = ekin + epot + eint,  mu = ekin + epot + 2 eint
 *   rms[a] = sqrt(dV sum x_a^2 |psi|^2 / norm)   (0 for absent axes)          */
typedef struct {
    double norm, mu, energy, ekin, epot, eint, rms[3];
} gp_obs;

/* Read-only description of a plan (host data). */
typedef struct {
    int ndim;
    int64_t n[3];
    int window[3];        /* truncation window K per axis: a value K points away is neglected
                             after decaying by rho^(K+1); -1 = exact solve */
    double rho[3];        /* max |c'_i| of the Thomas recurrence per axis */
    double window_bound[3]; /* rho^(K+1): bound on the window's relative truncation */
    int64_t step;         /* index of the next step (selects the trap schedule) */
    int64_t device_bytes; /* device memory owned by the plan */
    int xy_fused;         /* 3D: row segments per plane of the fused x+y sweep, 0 = separate sweeps */
} gp_plan_info;

typedef struct gp_plan gp_plan;
typedef struct gp_batch gp_batch;

/* Trap symmetries ("Nature of problem": besides 1d and fully anisotropic 2d/3d
 * traps, circularly symmetric 2d, spherically symmetric 3d and axially
 * symmetric 3d traps, which reduce the dimension). */
typedef enum { GP_CARTESIAN = 0, GP_CIRCULAR = 1, GP_SPHERICAL = 2, GP_AXIAL = 3 } gp_geometry;

/* ------------------------------------------------------------ core path */

/* Create a plan for an ndim-dimensional grid n[0..ndim) (x first) with
 * spacings dx[0..ndim), time step dt > 0, mode, trap (may be NULL: all
 * omega = 0), nonlinearity g and precision.  The problem is the paper's
 * "Nature of problem" (GP equation in 1d, 2d or 3d in a fully anisotropic
 * harmonic trap) discretised as in "Solution method" (split-step
 * Crank-Nicolson, imaginary- or real-time propagation).  Precomputes the
 * per-axis Thomas coefficients of the Crank-Nicolson substeps in FP64 on the
 * host (rounded once to FP32 for GP_C64) and allocates the plan's device
 * buffers on the current device (the plan owns them).
 * Errors: GP_EINVAL (ndim not 1..3, n < 1, dx <= 0, dt <= 0 or non-finite, bad
 * enum, bad schedule), GP_ENOMEM, GP_EHIP (no usable device). */
gp_status gp_plan_create(gp_plan **out, int ndim, const int64_t *n, const double *dx, double dt,
                         gp_mode mode, const gp_trap *trap, double g, gp_prec prec);

/* Create a plan for a symmetric trap ("Nature of problem"): GP_CIRCULAR
 * (2d, psi(r)), GP_SPHERICAL (3d, psi(r)) -- n[0] radial points, dx[0] = dr,
 * trap->omega[0] the radial frequency -- or GP_AXIAL (3d, psi(rho, z)) --
 * n = {N_rho, N_z}, dx = {drho, dz}, omega = {w_rho, w_z}; the wavefunction is
 * (N_z, N_rho) with rho fastest.  Radial points sit at r_i = (i + 1/2) dr, the
 * wall is a zero ghost at i = N, and the radial Crank-Nicolson substep uses the
 * finite-volume Laplacian with face areas r^(d-1) and exact cell volumes w_i as
 * weights (self-adjoint in sum w conj(u) v, so real time conserves the norm);
 * the axial z substep is the Cartesian one.  norm = m sum w |psi|^2 with
 * m = 2 pi dr, 4 pi dr, 2 pi drho dz.  gp_step and gp_observables work on the
 * plan (rms[0] = sqrt(<r^2>), rms[1] = sqrt(<z^2>) for axial); the adjoint and
 * batched forms do not.  Errors: GP_EINVAL as gp_plan_create and for a bad
 * geometry; GP_EUNSUPPORTED for GP_C64 or N_r (N_rho) above 1024. */
gp_status gp_plan_create_sym(gp_plan **out, gp_geometry geom, const int64_t *n, const double *dx, double dt,
                             gp_mode mode, const gp_trap *trap, double g, gp_prec prec);

/* Free the plan and its device buffers (NULL is allowed). */
gp_status gp_plan_destroy(gp_plan *plan);

/* Advance psi (device, in place, layout above) by nsteps >= 0 SSCN steps on
 * `stream`; asynchronous.  One step is the split-step Crank-Nicolson step of
 * "Solution method" as spelled out at the top of this file; imaginary-time
 * propagation (stationary states) returns psi with unit norm, real-time
 * propagation (dynamics) conserves it.  The plan's step index advances by
 * nsteps.  psi stays owned by the caller; the plan's work grid and partial
 * buffers are used as scratch.  Errors: GP_EINVAL (NULL plan/psi, nsteps < 0),
 * GP_EHIP (launch failure, or an earlier asynchronous fault). */
gp_status gp_step(gp_plan *plan, void *psi, int64_t nsteps, void *stream);

/* Observables of psi (device) into *out (host): the energy, chemical
 * potential and rms sizes that "Summary of revisions" lists among the
 * programs' outputs, plus the norm and the energy's parts (definitions at
 * gp_obs).  The trap is the one of the last step taken (step index - 1; a
 * schedule may change it), or of step 0 before any step.  FP64 accumulation
 * in a fixed order, so results are reproducible bit for bit.  Synchronises
 * `stream`.  Returns GP_ENONFINITE (with *out filled) if norm or energy is not
 * finite; GP_EINVAL for NULL arguments. */
gp_status gp_observables(gp_plan *plan, const void *psi, gp_obs *out, void *stream);

/* Set / get the index of the next step.  Setting it resumes a run from a
 * stored wavefunction -- the hand-over "Summary of revisions" describes, where
 * real-time programs read a wavefunction precomputed in imaginary time (NSTP
 * set to zero) -- or restarts a segment of the adjoint's checkpointed
 * recomputation; the index selects the trap schedule entry of each step.
 * GP_EINVAL for a NULL plan or a negative index. */
gp_status gp_plan_set_step(gp_plan *plan, int64_t step);
gp_status gp_plan_get_info(const gp_plan *plan, gp_plan_info *info);

/* 3D forward steps: enable (1 or 2, the default 2) or disable (0) the fused x+y
 * sweep.
 * The x and y Crank-Nicolson substeps of the step (program summary, "Solution
 * method") act plane by plane, so where the plan's shape allows (x extent 128,
 * 192 or 256, and a y window of 2..4 blocks that fits in LDS) one kernel reads
 * each xy-plane once and writes the result of both substeps; otherwise, or
 * when disabled, the sweeps run as separate kernels.  enable = 2 (the default)
 * keeps the y solver's elimination window in registers and double-buffers the
 * row tile; enable = 1 keeps the window in LDS.  Every choice gives the same
 * step up to rounding.  GP_EINVAL for a NULL plan or a flag outside 0..2. */
gp_status gp_plan_set_xy_fusion(gp_plan *plan, int enable);

/* Host-only (no GPU needed): one axis's Thomas table exactly as a plan stores
 * it, for checking.  The CN substep along an axis of n points is solved in the
 * form scaled by 1/e (unit off-diagonals):
 *     tridiag(1, delta_p, 1) u' = beta_p u_p - (u_{p-1} + u_{p+1}),
 * factorised as y_p = (rhs_p - y_{p-1}) c'_p, u'_p = y_p - c'_p u'_{p+1}, where
 * c'_0 = e/b, c'_p = e/(b - e c'_{p-1}) are rounded to the precision and
 * delta_p = 1/c'_p + c'_{p-1} is what the rounded values multiply out to;
 * beta_p = -conj(delta_p) in real time, -2/r - delta_p in imaginary time
 * (r = dt/(4 dx^2)).  Outputs, for p = 0..n-1: c[2p], c[2p+1] = c'_p and
 * beta[2p], beta[2p+1] = beta_p (interleaved complex, conjugated if adjoint),
 * *window = back-substitution window K (-1: exact two-pass solver), *rho =
 * max |c'_p|. */
gp_status gp_thomas_table(int64_t n, double dx, double dt, gp_mode mode, gp_prec prec, int adjoint,
                          double *c, double *beta, int *window, double *rho);

/* --------------------------------------------------- physical inputs (host) */
/* "Summary of revisions": the programs take physical inputs (number of atoms,
 * scattering length, oscillator length, trap anisotropy) and compute the
 * dimensionless nonlinearity from them.  In units of the oscillator length
 * l = sqrt(hbar / (m w)) and of hbar w, the 3d equation has g = 4 pi N a / l.
 * A tight confinement integrates out: in 2d (z frequency lambda w) g is
 * multiplied by the integral of the z ground state's |zeta|^4,
 * sqrt(lambda / (2 pi)); in 1d (transverse frequency nu w) by the transverse
 * ground state's, nu / (2 pi).  a in Bohr radii (5.29177210903e-11 m), l in
 * micrometres, confine = lambda (ndim 2) or nu (ndim 1), ignored in 3d.
 * GP_EINVAL for non-finite or out-of-range inputs or a NULL output. */
gp_status gp_nonlinearity(int ndim, double natoms, double a_bohr, double l_micron, double confine, double *g);

/* Oscillator length sqrt(hbar / (m 2 pi f)) in micrometres for an atomic mass
 * in atomic mass units and a trap frequency f in Hz (CODATA hbar and u). */
gp_status gp_osc_length(double mass_amu, double freq_hz, double *l_micron);

const char *gp_strerror(gp_status s);
const char *gp_last_error(void);

/* ------------------------------------------------------ adjoint form */

/* `nsteps` real-time steps of psi in place (as gp_step), storing the input of
 * each: states (device, nsteps consecutive grids of psi's precision and
 * layout, caller-owned) receives states[k] = psi before step (current step
 * index) + k.  This is what gp_step_adjoint consumes; a recomputed segment of
 * the checkpointed reverse sweep is one call.  Real-time plans only
 * (GP_EUNSUPPORTED otherwise).  Asynchronous. */
gp_status gp_step_record(gp_plan *plan, void *psi, int64_t nsteps, void *states, void *stream);

/* Reverse of `nsteps` real-time steps n_first .. n_first+nsteps-1, in the
 * gradient convention G = dL/dRe + i dL/dIm (PyTorch's for a real loss).
 *   states : device, nsteps consecutive wavefunctions; states[k] is the INPUT
 *            of step n_first + k (same precision/layout as psi)
 *   lambda : device, in place: on entry G of the output of the last step, on
 *            return G of the input of step n_first
 *   dsched : device FP64[nsteps] or NULL: dsched[k] = dL/d omega_s(n_first+k)
 *            for the schedule axis s (written, not accumulated)
 *   dg     : device FP64[1] or NULL: dL/dg accumulated (+=) over the steps
 * Per step n, with u the output of the potential substep and lambda_u its
 * gradient (obtained by the conjugate Crank-Nicolson solves z, y, x):
 *   w = Im(conj(lambda_u) u),  lambda_psi = e^{i theta} lambda_u + 2 dt g w psi,
 *   dL/d omega_s(n) = dt omega_s(n) sum w x_s^2,   dL/dg += dt sum w |u|^2.
 * Real-time plans only (GP_EUNSUPPORTED otherwise).  Asynchronous. */
gp_status gp_step_adjoint(gp_plan *plan, const void *states, void *lambda, int64_t n_first,
                          int64_t nsteps, double *dsched, double *dg, void *stream);

/* ------------------------------------------------------ batched form */

/* A batch of `count` independent 2D problems (problem k: grid n[2k], n[2k+1]
 * (x first, each 1..1024), spacing dx[k] on both axes, step dt[k], trap
 * traps[k].omega[0..1] (static: a schedule gives GP_EUNSUPPORTED), nonlinearity
 * g[k]), all in one mode and precision -- many of the paper's 2d problems
 * ("Nature of problem") advanced by one call.
 * Each problem gets a plan as from gp_plan_create; the batch advances them
 * together (gp_batch_step), either with two launches per step (all problems'
 * x sweeps, then all y sweeps) or, in real time, with one persistent launch
 * for all steps whose wavefronts take (step, phase, problem, tile) items from
 * a device queue and wait on per-problem completion counters.
 * Errors: GP_EINVAL, GP_ENOMEM, GP_EHIP; GP_EUNSUPPORTED for a problem the
 * batched kernels do not run (a y sweep that needs the exact two-pass solver
 * or a window deeper than 8 blocks of 4 points, i.e. dt/dx^2 too large, or
 * rings beyond the device's LDS). */
gp_status gp_batch_create(gp_batch **out, int count, const int64_t *n /* [count][2] */,
                          const double *dx, const double *dt, gp_mode mode,
                          const gp_trap *traps /* [count] */, const double *g, gp_prec prec);
gp_status gp_batch_destroy(gp_batch *batch);

/* Advance every problem k (psis[k]: device grid of problem k, layout as
 * gp_step's) by nsteps steps; the pointer array is host memory.  Imaginary
 * time renormalises every problem to unit norm.  Asynchronous, except that a
 * persistent launch synchronises `stream` to read its error flag: a bounded
 * device-side dependency wait that gave up yields GP_ETIMEOUT; the grids'
 * contents are then undefined (some items ran, some did not) and the step
 * indices are left unchanged, so the caller must reload them. */
gp_status gp_batch_step(gp_batch *batch, void *const *psis, int64_t nsteps, void *stream);

/* Time candidate configurations -- persistent or phased launch, lines per work
 * item (1, 2, 4), y segments per line (1..32, capped per problem by the
 * segments its y window allows), persistent grid size (256..2048 workgroups)
 * -- for 10 steps each on scratch copies of the problems and keep the fastest;
 * then, per line length (each side length of the problems, those carrying the
 * most points first), try 1, 2, 4 and 8 lines per item and, for y lines solved
 * by the windowed solver, 1..32 segments, keeping a change when it is at least
 * 1% faster.  cache_path (may be NULL): text file of previous results, one line
 * "key persistent lines ysegs grid [sides len:lines:ysegs ...]" per batch shape
 * (key: the precision, mode and sorted problem sizes); read first, appended to.
 * Synchronises `stream`. */
gp_status gp_batch_autotune(gp_batch *batch, const char *cache_path, void *stream);

/* gp_batch_autotune on the null stream (the boundary's tuning call). */
gp_status gp_autotune(gp_batch *batch, const char *cache_path);

/* Bound, in polls (each a short sleep), of one dependency wait in the
 * persistent launch (default 2^22, about 0.3 s): for callers that must bound a
 * stalled launch, and for exercising the GP_ETIMEOUT path. */
gp_status gp_batch_set_wait_limit(gp_batch *batch, uint32_t polls);

/* Read / set the configuration explicitly (persistent = 1 needs real time;
 * lines 1..64, ysegs 1..64, grid 1..65536; GP_EINVAL outside).  lines and
 * ysegs are the defaults for every line length; setting them clears the
 * per-length settings below. */
gp_status gp_batch_get_config(const gp_batch *batch, int *persistent, int *lines, int *ysegs, int *grid);
gp_status gp_batch_set_config(gp_batch *batch, int persistent, int lines, int ysegs, int grid);

/* Per line length `side` (points on a line: a problem's nx for its x lines,
 * its ny for its y lines): lines per work item and y segments (1..64 each)
 * used instead of the defaults for the lines of that length.  get returns the
 * values in effect for `side`.  GP_EINVAL for side < 1, a NULL pointer or
 * values outside 1..64. */
gp_status gp_batch_set_side_config(gp_batch *batch, int64_t side, int lines, int ysegs);
gp_status gp_batch_get_side_config(const gp_batch *batch, int64_t side, int *lines, int *ysegs);

/* Observables of problem k of a batch (as gp_observables).  GP_EINVAL for a
 * NULL batch or k outside 0..count-1. */
gp_status gp_batch_observables(gp_batch *batch, int k, const void *psi, gp_obs *out, void *stream);

/* -------------------------------------------------------- density outputs */
/* "Summary of revisions" lists the programs' density outputs: the condensate
 * density, reduced (integrated) 1d and 2d densities, and in the real-time
 * programs the rms sizes as the dynamics evolves after a perturbation.  These
 * compute them on the device beside the step; out buffers are caller-owned
 * device FP64 arrays; every call is asynchronous on `stream`. */

/* out[p] = |psi_p|^2 at every grid point p (plan layout, npts values).
 * GP_EINVAL for NULL arguments. */
gp_status gp_density(gp_plan *plan, const void *psi, double *out, void *stream);

/* |psi|^2 integrated over every axis whose bit is clear in keep_mask (bit a =
 * axis a, x = bit 0), by rectangle sums in a fixed order; out holds the kept
 * axes' grid, x fastest -- e.g. keep_mask 4 on a 3D plan gives
 * n(z_k) = sum_{i,j} |psi_ijk|^2 dx dy (npts / (nx ny) values).  Cartesian plans
 * of 2 or 3 dimensions and axial plans; for an axial plan integrating rho
 * carries the weights 2 pi r_i drho (keep z: the linear density n(z), summing
 * to the norm with dz) and integrating z gives the column density of each rho.
 * A two-axis integration leaves its intermediate in the plan's work grid.
 * GP_EINVAL for NULL arguments, a mask that keeps no axis or all of them, or a
 * 1D (including circular / spherical) plan. */
gp_status gp_density_reduced(gp_plan *plan, const void *psi, int keep_mask, double *out, void *stream);

/* Advance psi by nsteps steps exactly as gp_step, in blocks of `every` steps,
 * recording the observables of the state before the first block and after
 * every block: out (device) receives nsteps/every + 1 records of
 * GP_SERIES_FIELDS FP64 values -- step index, norm, mu, energy, ekin, epot,
 * eint, rms[0], rms[1], rms[2] (as gp_obs) -- with no host synchronisation.
 * GP_EINVAL unless nsteps is a non-negative multiple of every >= 1. */
#define GP_SERIES_FIELDS 10
gp_status gp_step_series(gp_plan *plan, void *psi, int64_t nsteps, int64_t every, double *out, void *stream);

/* --------------------------------------- observables without allocation */

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * observables of gp_observables for a grid described by its arguments instead
 * of a plan (ndim, n[], dx[] as gp_plan_create; omega[ndim] the trap, NULL for
 * none; psi device, layout above; *out host).  Same kernels and summation
 * order as gp_observables, so the results are bitwise those of a plan of that
 * grid and trap.  The partial sums live in one static device array of the
 * library per device ((GP_OBS_NOALLOC_MAX_GROUPS + 1) x 10 FP64, about
 * 640 KiB), looked up on the first call on a device; the call allocates
 * nothing.  Every call on a device shares that array, so calls that overlap on
 * one device (other threads, other streams) race.  Synchronises `stream`.
 * Errors: GP_EINVAL (bad argument), GP_EUNSUPPORTED (grid needs more than
 * GP_OBS_NOALLOC_MAX_GROUPS workgroups: ceil(nx/64) ceil(ny/16) above it, e.g.
 * a 2D grid beyond 2048 x 4096 or a 1D grid beyond 524288 points), GP_EHIP,
 * GP_ENONFINITE. */
#define GP_OBS_NOALLOC_MAX_GROUPS 8192
gp_status gp_observables_noalloc(int ndim, const int64_t *n, const double *dx, const double *omega, double g,
                                 gp_prec prec, const void *psi, gp_obs *out, void *stream);

/* ---------------------------------------------------- measurement aids */

/* Per-kernel timing with HIP events recorded on the plan's launch stream around
 * every kernel launch; capacity = number of launches to record (0 disables). */
gp_status gp_plan_timing_enable(gp_plan *plan, int64_t capacity);

/* Synchronise the events and report, per kernel kind (names in
 * gp_kernel_name(kind), kind = 0..GP_NUM_KERNEL_KINDS-1), the number of
 * recorded launches and their total duration in milliseconds; clears the log. */
#define GP_NUM_KERNEL_KINDS 15
gp_status gp_plan_timing_read(gp_plan *plan, int64_t *counts, double *total_ms);
const char *gp_kernel_name(int kind);

/* Plain device copy of `bytes` (multiple of 16) from src to dst: the
 * reference kernel for bandwidth and counter calibration.  Asynchronous. */
gp_status gp_copy_probe(void *dst, const void *src, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GP_H */
