/*
 * sscn.h -- C ABI of the MI355X (gfx950) split-step Crank-Nicolson (SSCN)
 * Gross-Pitaevskii propagator.
 *
 * The operation (the paper's program summary, "Nature of problem" and
 * "Solution method"): the time-dependent GP equation for a condensate with
 * contact interaction in a harmonic trap, in one, two or three dimensions,
 * is discretised in space and time and propagated over small time steps by
 * the split-step Crank-Nicolson method, in imaginary time (stationary
 * states) or real time (dynamics).  In the dimensionless form used here
 *
 *     i dpsi/dt = [ -1/2 Lap + V + g |psi|^2 ] psi,
 *     V = (omega_x^2 x^2 + omega_y^2 y^2 + omega_z^2 z^2) / 2,
 *
 * one step of length dt is: the pointwise substep
 *     psi <- exp(-dt (V + g|psi|^2)) psi          (imaginary time)
 *     psi <- exp(-i dt (V + g|psi|^2)) psi        (real time),
 * then, along x, y, z in turn, the Crank-Nicolson kinetic substep
 *     (1 + s T) v = (1 - s T) u,  T = tridiag(-1, 2, -1),
 *     s = dt/(4 dx_a^2) (imaginary) or i dt/(4 dx_a^2) (real),
 * with psi = 0 just outside the grid; in imaginary time the state is then
 * renormalised to dV * sum |psi|^2 = 1 (every `renorm_every` steps).
 *
 * Grid: axis a has n_a points at x_a(i) = (i - (n_a - 1)/2) dx_a; unused axes
 * (a >= dim) have n_a = 1.  Layout: x fastest, p = i + n_x (j + n_y k).
 *
 * Symmetric traps ("Nature of problem": circular symmetry in 2D, radial and
 * axial symmetry in 3D; geom below).  Circular (2D) and spherical (3D):
 * psi(r), one stored axis (dim = 1); axial (3D): psi(rho, z), two stored
 * axes (dim = 2, axis 0 rho, axis 1 z).  The radial axis has n_0 cells
 * [i dr, (i+1) dr] with values at r_i = (i + 1/2) dr; its Laplacian
 * (1/r^k) d/dr (r^k d/dr), k = 1 (circular, axial) or 2 (spherical), is the
 * finite-volume form
 *     (Lap psi)_i = [F_{i+1} (psi_{i+1} - psi_i) - F_i (psi_i - psi_{i-1})] / (W_i dr^2)
 * with face weights F_i = (i dr)^k (F_0 = 0: no flux through the origin)
 * and cell weights W_i = r_i (k = 1) or r_i^2 + dr^2/12 (k = 2); psi = 0
 * past the outer edge.  z is a Cartesian axis as above.  Inner product and
 * norm: c dr (dz) sum W_i conj(a) b, c = 2 pi (circular, axial) or 4 pi
 * (spherical).  A step is the pointwise substep with V = omega_0^2 r^2/2
 * (+ omega_1^2 z^2/2, axial), then the Crank-Nicolson substep
 * (1 + tau H_r) v = (1 - tau H_r) u along r, H_r = -Lap_r/2, tau = dt/2 or
 * i dt/2 (a general tridiagonal system per radial line), then (axial) along
 * z as on a Cartesian axis; in imaginary time the renormalisation in this
 * norm.  Observables are those of this Hamiltonian in this inner product;
 * mean/msq hold <r>, <r^2> (axis 0) and <z>, <z^2> (axis 1, axial).
 * State dtype by (mode, prec):
 *     IMAG + F64 -> double        IMAG + F32 -> float
 *     REAL + F64 -> double2 (re, im interleaved, like complex128)
 *     REAL + F32 -> float2  (complex64)
 * In the F32 forms the state, the pointwise substep and the line sweeps are
 * FP32; the Thomas coefficient tables, the norm, the renormalisation and all
 * observables stay FP64.
 *
 * Conventions.  0 is success, negative values are errors, positive values
 * are informational.  Every argument is validated before any side effect.
 * No C++ exception or abort crosses this boundary.  A handle is not thread
 * safe; several handles may share one stream.  The library allocates no
 * device memory: the caller owns the state and the workspace (device
 * pointers) and the HIP stream (a hipStream_t passed as void*, NULL = the
 * null stream), all of which must outlive the handle.
 */
#ifndef SSCN_H
#define SSCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSCN_ABI_VERSION 2

/* status codes */
#define SSCN_OK              0
#define SSCN_NOT_CONVERGED   1   /* informational: step cap reached first */
#define SSCN_BUSY            2   /* informational: results not ready yet (non-blocking poll) */
#define SSCN_E_INVALID      -1   /* bad argument or problem */
#define SSCN_E_HIP          -2   /* a HIP runtime call failed */
#define SSCN_E_NONFINITE    -3   /* norm or chemical potential is NaN/Inf */
#define SSCN_E_NOSPACE      -4   /* slot busy / buffer too small */
#define SSCN_E_UNSUPPORTED  -5   /* valid problem outside the library's limits */

/* mode and precision */
#define SSCN_IMAG 0
#define SSCN_REAL 1
#define SSCN_F64  0
#define SSCN_F32  1

/* trap geometry (sscn_problem.geom) */
#define SSCN_GEOM_CART 0   /* anisotropic trap on a Cartesian grid of dim axes */
#define SSCN_GEOM_CIR  1   /* 2D circular symmetry: psi(r), dim = 1 */
#define SSCN_GEOM_SPH  2   /* 3D spherical symmetry: psi(r), dim = 1 */
#define SSCN_GEOM_AXI  3   /* 3D axial symmetry: psi(rho, z), dim = 2 */
#define SSCN_RADIAL_MAX 16384   /* longest radial axis (cells) */

typedef struct {
    int32_t dim;            /* 1, 2 or 3 */
    int32_t n[3];           /* points per axis; axes >= dim must be 1 */
    double  dx[3];          /* spacing per axis (> 0 for axes < dim) */
    double  omega[3];       /* trap frequencies (>= 0) */
    double  g;              /* nonlinearity used by the propagation */
    double  dt;             /* time step (> 0) */
    int32_t mode;           /* SSCN_IMAG or SSCN_REAL */
    int32_t prec;           /* SSCN_F64 or SSCN_F32 */
    int32_t renorm_every;   /* IMAG: >= 1 (renormalise every k steps); REAL: 0 */
    int32_t observe_every;  /* >= 0; observation interval of sscn_run / batch */
    int32_t geom;           /* SSCN_GEOM_*; 0 (Cartesian) for a zero-filled struct */
    int32_t pad_;           /* 0 */
} sscn_problem;

typedef struct {
    int64_t step;           /* steps taken since create */
    double  norm;           /* dV sum |psi|^2 */
    double  mu;             /* (K + P + g I) / norm */
    double  energy;         /* (K + P + g I / 2) / norm */
    double  ekin;           /* K = 1/2 dV sum_a sum_edges |dpsi|^2 / dx_a^2 */
    double  epot;           /* P = dV sum V |psi|^2 */
    double  eint;           /* I = dV sum |psi|^4 */
    double  mean[3];        /* <x_a> */
    double  msq[3];         /* <x_a^2> */
    int32_t status;         /* SSCN_OK or SSCN_E_NONFINITE */
    int32_t pad_;
} sscn_obs;

typedef struct sscn_solver sscn_solver;

/* Physical inputs of a condensate ("Reasons for the new version" and
 * "Summary of revisions": the programs take the number of atoms, the
 * scattering length and the oscillator length of the trap, and compute the
 * dimensionless nonlinearity they propagate with). */
typedef struct {
    int32_t dim;            /* 1, 2 or 3: dimensions of the propagated problem */
    int32_t pad_;           /* 0 */
    double  atoms;          /* N > 0 */
    double  scattering_length;  /* a, in Bohr radii (any sign) */
    double  mass;           /* atomic mass, in unified atomic mass units (> 0) */
    double  omega;          /* reference angular trap frequency (rad/s, > 0): time unit 1/omega,
                               length unit l = sqrt(hbar / (m omega)) */
    double  tight[2];       /* frozen directions' trap frequencies over omega (> 0):
                               dim 2: tight[0] (z); dim 1: tight[0], tight[1] (y, z); dim 3: unused */
} sscn_units;

/* Calls that carry no operation of the paper (version, status text, sizes,
 * timing, tile hints, plan queries, batching and its admission) are marked
 * "systems call" below: they serve the measurement, the autotuner and the
 * batched serving loop built around the method.  Every other call cites the
 * passage of the paper's program summary that defines what it computes. */

/* "Reasons for the new version", "Summary of revisions" (physical inputs ->
 * the dimensionless nonlinearity).  Host only.  In units of l and 1/omega
 * the 3D equation has g = 4 pi N a / l; a problem of lower dimension is the
 * 3D one with the frozen directions in their oscillator ground states
 * (widths d = 1/sqrt(tight)), integrated out:
 *     dim 3: g = 4 pi N a / l
 *     dim 2: g = 4 pi N a / l * sqrt(tight[0] / (2 pi))
 *     dim 1: g = 4 pi N a / l * sqrt(tight[0] tight[1]) / (2 pi)
 * (the factors are the integrals of the frozen Gaussians' fourth power).
 * The paper prints no formula; these are the standard reductions.  Writes g
 * and, when non-NULL, l in metres and 1/omega in seconds.  SSCN_E_INVALID
 * for a NULL pointer, dim out of range or a non-positive / non-finite
 * input. */
int sscn_units_to_g(const sscn_units *u, double *g, double *length_m, double *time_s);

/* Systems call: SSCN_ABI_VERSION of the loaded library. */
int sscn_abi_version(void);

/* Systems call: static text for a status code (never NULL). */
const char *sscn_status_string(int status);

/* Host-only check of a problem (no GPU access).  The problem is the one of
 * "Nature of problem": the GP equation in one, two or three dimensions in a
 * harmonic trap, given by its grid, trap frequencies, nonlinearity, time step
 * and imaginary/real-time mode.  SSCN_E_INVALID if dim is
 * not 1..3, an n_a < 1, n_a != 1 on an unused axis, dx_a <= 0 or non-finite
 * on a used axis, omega < 0 or non-finite, g non-finite, dt <= 0 or
 * non-finite, mode/prec out of range, renorm_every < 1 in IMAG or != 0 in
 * REAL, observe_every < 0, geom out of range, dim != 1 for the circular
 * and spherical traps or != 2 for the axial trap.  SSCN_E_UNSUPPORTED if
 * the grid exceeds this build's limits (more than 2^40 points, or a radial
 * axis of more than SSCN_RADIAL_MAX cells). */
int sscn_validate(const sscn_problem *pb);

/* Systems call (admission by HBM footprint).
 * Bytes of the caller-owned state (points * element size) and workspace.
 * The workspace holds the FP64 Thomas tables, reduction partials and device
 * scalars; the two sums are what a solve keeps resident in HBM. */
int sscn_state_bytes(const sscn_problem *pb, size_t *bytes);
int sscn_workspace_bytes(const sscn_problem *pb, size_t *bytes);

/* "Solution method" (discretisation in space and time): bind a solver to
 * caller memory: d_psi (state, layout above, at least
 * sscn_state_bytes), d_ws (workspace, at least sscn_workspace_bytes, 256-byte
 * aligned), hip_stream.  Precomputes the FP64 Thomas tables of every axis on
 * the host and uploads them to d_ws on the stream (the call waits for that
 * copy).  The state is not touched.  Errors: SSCN_E_INVALID (bad problem,
 * NULL pointer, misaligned workspace), SSCN_E_HIP. */
int sscn_create(const sscn_problem *pb, void *d_psi, void *d_ws, void *hip_stream,
                sscn_solver **out);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same as
 * sscn_create, but the workspace is the library's own static device array
 * of SSCN_STATIC_WS_BYTES bytes on the current device (the device the
 * stream belongs to), which each GPU the library runs on holds until the
 * process ends.  The call allocates no device or pinned host memory (no
 * hipMalloc, hipHostMalloc or hipFree; the handle and the host image of the
 * tables are ordinary host memory).  It rewrites the whole array (tables,
 * then zeros), so nothing of an earlier solver's contents survives; it
 * waits for that copy.  One live solver per device may hold the array:
 * while one does, another call on that device returns SSCN_E_NOSPACE;
 * sscn_destroy releases it after waiting for the solver's stream.  Every
 * later call on the solver is the same as on one from sscn_create; calls
 * on it from several threads at once race, as for any handle.  Errors as
 * sscn_create, plus SSCN_E_UNSUPPORTED when the problem's workspace
 * (sscn_workspace_bytes) exceeds SSCN_STATIC_WS_BYTES or the device index
 * is 64 or more, SSCN_E_NOSPACE as above, SSCN_E_HIP if the array's device
 * address cannot be taken. */
#define SSCN_STATIC_WS_BYTES ((size_t)4 << 20)
int sscn_create_noalloc(const sscn_problem *pb, void *d_psi, void *hip_stream, sscn_solver **out);

/* "Solution method" (propagation in imaginary or real time over small time
 * steps): enqueue nsteps >= 0 SSCN steps on the stream and return.  When the
 * stream reaches the end of the call the state is complete: in imaginary
 * time it is renormalised if the last step was a renormalisation step.  On a
 * stream other than the legacy default stream the call replays hipGraphs of
 * 32, 16, 8, 4, 2 and 1 steps (the binary decomposition of nsteps), each
 * captured on first use and kept per (length, renormalisation pattern);
 * sscn_set_g and sscn_destroy drop them.  The kernels and results are those
 * of direct launches. */
int sscn_step(sscn_solver *s, int64_t nsteps);

/* Systems call: capture now, without launching any kernel, the graphs that
 * a following sscn_step(s, nsteps) from the current step will replay, and
 * upload them to the device on the stream, so that call does no capture or
 * upload of its own (a timed region, a latency-bound loop).  Never
 * required: sscn_step captures what is missing.  SSCN_E_HIP if an upload
 * fails. */
int sscn_prepare(sscn_solver *s, int64_t nsteps);

/* "Summary of revisions" (the general output file holds the energy and the
 * chemical potential; the dynamics files hold rms sizes): observables of the
 * current state, with the moments <x_a>, <x_a^2> from which the rms sizes
 * follow; waits for the stream.  Returns SSCN_E_NONFINITE (and fills out) if
 * the norm or mu is NaN or Inf. */
int sscn_observe(sscn_solver *s, sscn_obs *out);

/* "Solution method" and "Summary of revisions" (imaginary-time iterations
 * that yield the stationary state, with its energy and chemical potential
 * written out; real-time iterations with the rms sizes written per time):
 * propagate until |mu(t) - mu(t - observe_every)| < mu_tol at an observation
 * step (observe_every from the problem, >= 1), or until max_steps more steps
 * were taken.  Rows of the observation trace go to trace[0..trace_cap) and
 * their count to *rows (either may be NULL/0).  Returns SSCN_OK on
 * convergence, SSCN_NOT_CONVERGED at the cap, SSCN_E_NONFINITE if the state
 * blew up (the trace ends at that row).  Waits for the stream at every
 * observation, except with mu_tol == 0 (no convergence test, a fixed number
 * of steps): then the observations are queued behind the steps without
 * waits and read back once per 4096 of them, so after a blow-up the steps
 * of the rest of that group have also been taken (the step count in the
 * handle says how many).  Allocates pinned host memory for that mode. */
int sscn_run(sscn_solver *s, int64_t max_steps, double mu_tol, sscn_obs *trace,
             int64_t trace_cap, int64_t *rows);

/* "Summary of revisions" (the dynamics is generated by multiplying the
 * nonlinearity by a given factor during the real-time iterations, starting
 * from the imaginary-time state): change the nonlinearity for later steps
 * and observables (a quench).  SSCN_E_INVALID if g is not finite. */
int sscn_set_g(sscn_solver *s, double g);

/* Systems call (measurement).
 * Enqueue nsteps steps exactly as sscn_step does, with HIP events recorded
 * around every kernel, wait, and report the mean duration in milliseconds of
 * each kernel class over the steps in ms[0..SSCN_NKERNELS).  Classes: 0 the
 * pointwise + x sweep, 1 the y sweep, 2 the z sweep (+ norm partials),
 * 3 the norm finalisation, 4 the end-of-call scale pass; a class that did not
 * run reports 0.  Timing aid for the benchmark; results are those of
 * sscn_step. */
#define SSCN_NKERNELS 5
int sscn_step_timed(sscn_solver *s, int64_t nsteps, double *ms);

/* Systems call (autotuner).
 * Tile hints (used by the tuner; Cartesian traps only, SSCN_E_UNSUPPORTED
 * otherwise): for problems of pb's shape (dim, n, mode,
 * prec), use chunk[0] points per thread on x lines and chunk[1], chunk[2] on
 * y and z lines (powers of two <= 64; 0 keeps the default).  Applies to later
 * sscn_workspace_bytes / sscn_create calls of that shape, process-wide.
 * SSCN_E_INVALID for a bad problem or chunk, SSCN_E_UNSUPPORTED if a chunk
 * does not fit the register-resident kernels for that shape. */
int sscn_set_tile_hint(const sscn_problem *pb, const int32_t chunk[3]);
int sscn_clear_tile_hints(void);

/* Systems call (autotuner, tests).
 * Kernel plan of a problem, 8 ints per axis (x, y, z): kind (0 ROW: lanes
 * along the line, 1 COL: lanes across lines, 2 one-thread-per-line
 * fallback, 3 radial line per block, -1 unused axis), points per thread,
 * waves per line group (ROW), per block (COL) or per line (radial), lanes
 * per line (COL; ROW: lanes of a wave per line, 64, or 16 for lines of at
 * most 64 points taken four to a wave; 1 otherwise), grid size, block
 * size, first index of the constant tail of the Thomas table, and the scan
 * depth (ROW: shuffle steps; COL: preceding chunks folded).  info needs
 * cap >= 24 entries. */
int sscn_plan_info(const sscn_problem *pb, int32_t *info, int32_t cap);

/* Systems call: free the handle's host state (the caller's device memory is
 * untouched).
 * Waits for the stream. */
int sscn_destroy(sscn_solver *s);

/* Integrated densities (the paper's n_1D and n_2D outputs, integrating
 * |psi|^2 over the other axes): out is a caller-owned device buffer of
 * n[keep] doubles (1D) or of the two remaining axes' points in layout order
 * (2D, dim == 3 only).  Enqueued on the stream; FP64.  n_1D uses the
 * solver's workspace as scratch (stream-ordered with the steps, so it may
 * be called between sscn_step calls without a wait).  Cartesian traps
 * only: SSCN_E_UNSUPPORTED for the symmetric ones. */
int sscn_density_1d(sscn_solver *s, int keep, void *d_out);
int sscn_density_2d(sscn_solver *s, int drop, void *d_out);

/* ------------------------------------------------------------------------
 * Batched persistent stepping (many uneven instances, FP32 forms).
 *
 * Systems calls (batching): each instance is the problem of "Nature of
 * problem" propagated by the method of "Solution method" in imaginary or
 * real time, exactly as sscn_step would; what these calls add is many
 * instances per launch.
 *
 * A batch advances every running instance by one SSCN step per launch of a
 * persistent kernel whose blocks take tiles of all instances from a work
 * list in dependency order (x tiles, then y, z, observation tiles, then one
 * finalisation per instance); on a non-null stream a call's launches are
 * captured once into a hipGraph and replayed.  A 1D instance whose line
 * fits one block (a solo instance) takes whole steps inside one block and
 * may advance several steps per launch: 64 per launch while every instance
 * is solo; in a batch on a non-null stream that also holds larger
 * instances, a kernel of its own on a second stream (created with the
 * batch) steps the solo instances for as long as the call's persistent
 * launches run, at least once per call.  The steps taken are reported per
 * instance (sscn_batch_slot.steps); the arithmetic of a step is the same
 * either way.  Every instance uses the same
 * method as sscn_step with prec = SSCN_F32 and renorm_every = 1 (imaginary
 * time) and is observed every observe_every steps; a ground-state instance
 * stops at the first observation with |mu - mu_prev| < mu_tol (mu_tol > 0),
 * any instance stops after max_steps.  An instance's tile shapes depend only
 * on its own shape and all its reductions have fixed order, so its results
 * do not depend on the other instances.  The caller owns every device
 * buffer: the control block, and each instance's state and workspace.
 * ------------------------------------------------------------------------ */
typedef struct sscn_batch sscn_batch;

#define SSCN_SLOT_EMPTY     0
#define SSCN_SLOT_RUNNING   1
#define SSCN_SLOT_CONVERGED 2   /* |d mu| < mu_tol reached */
#define SSCN_SLOT_DONE      3   /* max_steps taken */
#define SSCN_SLOT_NONFINITE 4   /* norm or mu became NaN/Inf; the instance stopped */

typedef struct {
    int32_t  state;         /* SSCN_SLOT_* */
    int32_t  pad_;
    int64_t  steps;         /* steps taken since admission */
    double   last_norm;     /* dV sum |psi|^2 after the last step, before renormalisation */
    sscn_obs obs;           /* observables at the last observation step (obs.step) */
} sscn_batch_slot;

/* Bytes of the control block for max_slots instances and a work list of up
 * to max_items tiles per step.  SSCN_E_INVALID for out-of-range sizes. */
int sscn_batch_ctl_bytes(int32_t max_slots, int64_t max_items, size_t *bytes);

/* Bytes of one instance's workspace in a batch (FP64 tables and partials).
 * SSCN_E_UNSUPPORTED unless prec == SSCN_F32, geom == SSCN_GEOM_CART and
 * the lines fit the persistent kernel's tiles (x lines up to 16384 points in
 * float and complex; y and z lines up to 1024 (complex) / 2048 (float)
 * points). */
int sscn_batch_workspace_bytes(const sscn_problem *pb, size_t *bytes);

/* Batch tile hints (used by the tuner): for instances of pb's shape (dim, n,
 * mode), chunk[a] points per thread on axis a, 0 keeping the default choice.
 * x lines: 1, 2, 3, 4, 6, 8 (12, 16 in imaginary time), honoured only when
 * one wave covers the line; y and z lines: 2, 3, 4, 5, 6, 8 (10, 12, 16 in
 * imaginary time).  Applies to later admissions and plan queries of that
 * shape, process-wide; an admitted instance keeps its geometry, and the
 * geometry of an instance depends on its shape only.  SSCN_E_INVALID for a
 * bad problem or a chunk outside these lists. */
int sscn_batch_set_tile_hint(const sscn_problem *pb, const int32_t chunk[3]);
int sscn_batch_clear_tile_hints(void);

/* Geometry of pb's instances in the persistent kernel at the default split,
 * 8 ints per axis (x,
 * y, z): kind (0 ROW, 1 COL, -1 unused axis), points per thread, waves per
 * line (ROW) or per sub-tile (COL), lanes per line (COL; 1 otherwise), work
 * items per step, line groups (ROW) or sub-tile sets (COL) per item, scan
 * depth, and 1 when the instance needs the kernel variant for long lines.
 * info needs cap >= 24 entries.  Errors as sscn_batch_workspace_bytes. */
int sscn_batch_plan_info(const sscn_problem *pb, int32_t *info, int32_t cap);

/* Create a batch over a caller-owned, 256-byte aligned device control block
 * of at least sscn_batch_ctl_bytes bytes, on hip_stream.  Clears the block.
 * Allocates pinned host mirrors only (no device memory); on a non-null
 * stream it also creates one HIP stream and two events, released by
 * sscn_batch_destroy.  SSCN_E_HIP if any of these fails. */
int sscn_batch_create(int32_t max_slots, int64_t max_items, void *d_ctl, size_t ctl_bytes, void *hip_stream,
                      sscn_batch **out);

/* Work-item split of the batch: every pass of an instance is cut into items
 * of about (points / parts) grid points (at least 32K, at most 256K).  Each
 * item pays a claim, a dependency wait and a release, so fewer, larger
 * items (small parts) cost less per point when many instances fill the
 * device, and more, smaller ones (large parts) finish a few running
 * instances sooner.  Default 32; 1 <= parts <= 4096.  Only while the batch
 * holds no instance (SSCN_E_INVALID otherwise): an instance's geometry, and
 * so its results, depend only on its shape and this setting.  Workspace
 * sizes do not depend on it. */
int sscn_batch_set_split(sscn_batch *b, int32_t parts);

/* Admit an instance into an empty slot: d_psi holds its initial state (layout
 * and dtype as for sscn_create), d_ws is its workspace.  Uploads its FP64
 * tables and waits for the copy.  SSCN_E_NOSPACE if the slot is busy or the
 * work list would exceed max_items; SSCN_E_INVALID / SSCN_E_UNSUPPORTED as
 * above.  No side effect on error. */
int sscn_batch_admit(sscn_batch *b, int32_t slot, const sscn_problem *pb, void *d_psi, void *d_ws,
                     double mu_tol, int64_t max_steps);

/* Release a slot; in imaginary time the state is renormalised first (the
 * pending factor of its last step is applied).  Waits for the stream. */
int sscn_batch_evict(sscn_batch *b, int32_t slot);

/* Enqueue nsteps persistent launches (one step of every running non-solo
 * instance each; solo instances as described above) and an asynchronous
 * copy of the per-instance status to a pinned host mirror.  All work of
 * the call is ordered before that copy on the batch's stream. */
int sscn_batch_step(sscn_batch *b, int32_t nsteps);

/* Copy the status of slots 0..nslots-1 from the mirror written by the last
 * sscn_batch_step.  wait = 0: SSCN_BUSY if that copy has not landed yet;
 * wait != 0: waits for it. */
int sscn_batch_poll(sscn_batch *b, sscn_batch_slot *out, int32_t nslots, int32_t wait);

/* Nonzero *flag if a bounded wait inside the persistent kernel ever gave
 * up (bit 0; results of that launch are then invalid) or a solo instance
 * met the solo kernel without a form for its line (bit 1; it did not
 * advance); waits for the stream. */
int sscn_batch_error(sscn_batch *b, int32_t *flag);

/* Free the batch's host state (device buffers belong to the caller). */
int sscn_batch_destroy(sscn_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* SSCN_H */
