/*
 * fcns.h -- C ABI of the MI355X FC-Gram pseudospectral solver for
 * incompressible flow in a cuboid with two periodic directions (x, y) and one
 * walled direction (z), after Fontana, Bruno, Mininni & Dmitruk, "Fourier
 * Continuation method for incompressible fluids with boundaries" (2020).
 *
 * Problem (Sec. 2): dv/dt + (v.grad)v = -grad p + nu lap v + G x
 *                   [+ gamma theta z, Sec. 7],  div v = 0,
 *                   v = 0 (and theta = 0) at z = 0 and z = Lz,
 * periodic in x and y.  Grid: x_q = q Lx/nx, y_r = r Ly/ny,
 * z_s = s Lz/(nz-1) (nz counts both walls).
 *
 * Conventions shared by all calls
 *  - Pointers named in the signatures are DEVICE pointers unless a comment
 *    says HOST.  The caller owns every pointer it passes; the context copies
 *    what it keeps (the FC table) and owns all device state and scratch, which
 *    is allocated once by fcns_create.  No call below fcns_create allocates
 *    device memory (fcns_rk_graph creates its graph object on first use).
 *  - Physical fields are float64 arrays [nz][ny][nx] (x fastest); a vector
 *    field is 3 such arrays back to back (x, y, z components).
 *  - All work is enqueued on the HIP stream given to fcns_create and is
 *    asynchronous with respect to the host; results are complete once that
 *    stream is synchronized.  One context per stream; calls on one context
 *    must not overlap.
 *  - Errors are returned as status codes; fcns_last_error() gives a message.
 *    The library never aborts the process.
 */
#ifndef FCNS_H
#define FCNS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcns_ctx fcns_ctx;

typedef enum {
  FCNS_OK = 0,
  FCNS_EINVAL = -1,     /* bad argument, shape or unsupported size */
  FCNS_ENOMEM = -2,     /* device allocation failed in fcns_create */
  FCNS_EDEVICE = -3,    /* a HIP call or kernel launch failed */
  FCNS_ENONFINITE = -4, /* a non-finite value was found in the state */
  FCNS_ESTATE = -5,     /* call out of order (e.g. rk_step before set_state) */
  FCNS_ECANCELED = -6   /* a served request was cancelled */
} fcns_status;

enum { FCNS_FP64 = 0, FCNS_MIXED = 1 };

typedef struct {
  int32_t nx, ny, nz;   /* nx, ny even; nz includes both walls; nz + C even
                           (the continued length N' = nz + C, eq. k) */
  double lx, ly, lz;    /* box lengths */
  int32_t fc_d, fc_C;   /* matching points d and continuation points C (Sec. 3) */
  const double* fc_table; /* HOST: Q_r (d x d, column j = Gram polynomial j at
                             the d right matching points) followed by A_r (C x d,
                             column j = blend-to-zero extension of Gram
                             polynomial j at the C continuation points), both
                             row-major float64 (App. B).  Copied at create. */
  double nu;            /* kinematic viscosity */
  double forcing_x;     /* body force G along +x (channel mean pressure
                           gradient, Sec. 6); 0 for none */
  int32_t boussinesq;   /* 1: also carry theta (Sec. 7) */
  double kappa, gamma;  /* thermal diffusivity and buoyancy rate (Boussinesq) */
  int32_t rk_order;     /* o of the time-splitting RK (Sec. 4.4), 1..4; o = 1 is
                           the forward-Euler splitting of Sec. 4.1 */
  double filter_beta;   /* exponential filter (Sec. 4.3); 0 -> 16 ln 10 */
  double filter_2p;     /* filter order 2p; 0 -> 100 */
  int32_t precision;    /* FCNS_FP64, or FCNS_MIXED: rk_step evaluates the
                           nonlinear term in FP32 (the back transforms of the
                           state, the x and y FFTs, the products with FP32
                           accumulation, and their mixed-space arrays), while
                           the continued state, the FC extension (FP64 tables
                           and sums), the transforms of the RK combine that form
                           v*, and the pressure projection with its
                           homogeneous correction stay FP64.  The standalone
                           calls (fc_*, rhs_nonlinear, pressure_project,
                           get/set_state) are FP64 in both. */
  int32_t keep_pressure;/* 1: rk_step also keeps the pressure of its last stage
                           (one extra mixed-space field write per step) */
} fcns_problem;

/* Create a context: validates the problem, builds the FFT plans, copies the
 * FC table (forming M_r = A_r Q_r^T in extended precision on the host) and
 * allocates all device buffers.  hip_stream: a hipStream_t (NULL = default
 * stream).  On failure *out is NULL.  Limits: nx <= 512, ny <= 1024,
 * N' = nz + C <= 512, at most 12 radix stages per transform length. */
fcns_status fcns_create(const fcns_problem* prob, void* hip_stream, fcns_ctx** out);

/* Release all device memory of the context (synchronizes its stream). */
fcns_status fcns_destroy(fcns_ctx* ctx);

/* FC-Gram continuation of real lines (Sec. 3, eq. fc:continuation; App. B):
 * out[l*out_ls + s*out_ps] = in[l*in_ls + s*in_ps] for s < nz, and for
 * s = nz + i (i < C): sum_j M_r[i][j] f[nz-d+j] + sum_j M_l[i][j] f[j] with
 * M_l = J M_r J.  nlines >= 0 lines of the context's nz points.  in/out must
 * not overlap.  Strides are in elements. */
fcns_status fcns_fc_extend(fcns_ctx* ctx, const double* in, int64_t nlines, int64_t in_ps,
                           int64_t in_ls, double* out, int64_t out_ps, int64_t out_ls);

/* FC spectral derivative along z of real lines of nz points (Sec. 3 and the
 * derivative rule of Sec. 4.2): out = R IFFT[(i k~z)^order FFT(E f)] for
 * order 1 (Nyquist mode zeroed) and R IFFT[-kz^2 FFT(E f)] for order 2.
 * Line l point s at in[l*ls + s*ps]; out uses the same strides. */
fcns_status fcns_fc_derivative(fcns_ctx* ctx, int32_t order, const double* in, int64_t nlines,
                               int64_t ps, int64_t ls, double* out);

/* fcns_fc_derivative for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context; the transform's twiddle table and the continuation
 * matrix M_r = A_r Q_r^T are staged in a static device array of the library
 * (64 KiB of twiddles and 256 float64 of M per device, held until the
 * process ends) instead of context buffers.  nz, lz, fc_d, fc_C and
 * fc_table (HOST, the layout of fcns_problem.fc_table) describe the lines as
 * in fcns_problem; order, in, nlines, ps, ls, out as in fcns_fc_derivative;
 * hip_stream: the stream to enqueue on (NULL = default).  EINVAL for bad
 * sizes, N' = nz + C odd or above 512, C * d above 256, or a transform table
 * above the array.  Allocates nothing (host or device).  Calls that overlap
 * on one device (other host threads, or streams not ordered with each other)
 * race on the shared array; its contents are rewritten by every call. */
fcns_status fcns_fc_derivative_noalloc(int32_t nz, double lz, int32_t fc_d, int32_t fc_C,
                                       const double* fc_table, int32_t order, const double* in,
                                       int64_t nlines, int64_t ps, int64_t ls, double* out,
                                       void* hip_stream);

/* Advective term -(v.grad)v (and -(v.grad)theta when theta != NULL; needs a
 * Boussinesq context) from the FC-continued transform of v (Sec. 4.2:
 * derivatives in Fourier space, products in physical space, no padding).
 * filtered = 1 also applies the exponential filter of Sec. 4.3 to the result.
 * Outputs are physical fields like the inputs. */
fcns_status fcns_rhs_nonlinear(fcns_ctx* ctx, const double* v, const double* theta,
                               int32_t filtered, double* nl_v, double* nl_theta);

/* Pressure projection of a physical field v* with stage coefficient c > 0
 * (Sec. 4.2 and Sec. 4.4 steps 3-5): v_out = v* - grad phi, phi = c p, with the
 * inhomogeneous part solved in continued Fourier space and the homogeneous
 * part in closed form so that v_out.z = 0 at the walls.  gradp_wall
 * (nullable): tangential pressure gradient at the walls, float64
 * [2 walls (z=0, z=Lz)][2 comps (x, y)][ny][nx], in p units. */
fcns_status fcns_pressure_project(fcns_ctx* ctx, const double* v_star, double c, double* v_out,
                                  double* gradp_wall);

/* Set the state from physical fields (theta required iff Boussinesq); the
 * wall pressure gradient used by the first stage is reset to 0. */
fcns_status fcns_set_state(fcns_ctx* ctx, const double* v, const double* theta);

/* Advance nsteps steps of the o-stage time-splitting Runge-Kutta scheme of
 * Sec. 4.4 with time step dt (stage coefficients c_j = dt/(o-j+1); each stage
 * injects the wall gradient of the previous stage's pressure, which for o = 1
 * is the time-splitting Euler scheme of Sec. 4.1).
 * Every stage checks the new state (all fields, theta included) for NaN and
 * infinity on the device (a flag raised by the z back transform of the
 * stage).  In the default check mode FCNS_CHECK_SYNC the call waits for its
 * steps and returns FCNS_ENONFINITE when the flag is up; the state is then
 * undefined and stays flagged until set_state / set_spectral.  In
 * FCNS_CHECK_DEFERRED the call is asynchronous on the context stream and
 * fcns_check_finite reports later; FCNS_CHECK_OFF skips the report. */
fcns_status fcns_rk_step(fcns_ctx* ctx, double dt, int32_t nsteps);

enum { FCNS_CHECK_OFF = 0, FCNS_CHECK_SYNC = 1, FCNS_CHECK_DEFERRED = 2 };
/* Select how rk_step, rk_graph and batch_step report a non-finite state
 * (see fcns_rk_step).  EINVAL for an unknown mode. */
fcns_status fcns_set_finite_check(fcns_ctx* ctx, int32_t mode);
/* Synchronize the context stream and return FCNS_ENONFINITE if a step
 * enqueued so far left a non-finite state (FCNS_OK otherwise). */
fcns_status fcns_check_finite(fcns_ctx* ctx);
/* The flag without synchronizing (1: non-finite).  It lives in pinned
 * host-coherent memory that the kernels write directly, so it covers every
 * step whose work has completed (e.g. behind an event that has completed). */
int32_t fcns_nonfinite_flag(const fcns_ctx* ctx);

/* Batched stepping of n independent contexts (HOST arrays of n context
 * pointers, time steps and step counts): step k of every context is
 * enqueued before step k + 1 of any, each on its own context stream, so
 * problems of different shapes overlap on the device.  Each context's result
 * is bitwise its own fcns_rk_step, and each reports a non-finite state in its
 * own check mode (FCNS_ENONFINITE is returned if any context in
 * FCNS_CHECK_SYNC mode has one; fcns_last_error of that context says so).
 * Contexts must not share a stream for the overlap (sharing is correct, only
 * serial). */
fcns_status fcns_batch_step(fcns_ctx* const* ctxs, int32_t n, const double* dts,
                            const int32_t* nsteps);

/* One launch for several problems: a batch of n FP64 contexts (HOST array;
 * different shapes allowed, N' <= 288 each, the same rk_order) and their
 * time steps (HOST, copied).  fcns_batch_run advances every member nsteps
 * steps: each context's x and y passes run on its own stream, and in every
 * stage whose output buffer is not its input (both stages of o = 2) one
 * kernel runs the fused z pass (continuation, z transforms, RK combine,
 * projection, back transforms) of all members together, workgroup by
 * workgroup over their pencil groups, on a stream of the batch; each member
 * waits for it before its next pass.  Each member's result matches its own
 * fcns_rk_step with the fused z pass to rounding (the same per-workgroup
 * code).  The batch reads its members' parameters, tables and buffers at
 * every run (a member retuned or given new parameters is picked up).
 * Members report a non-finite state in their own check mode.  create
 * allocates the batch's descriptors, stream and events; run allocates
 * nothing. */
typedef struct fcns_batch fcns_batch;
fcns_status fcns_batch_create(fcns_ctx* const* ctxs, int32_t n, const double* dts,
                              fcns_batch** out);
fcns_status fcns_batch_run(fcns_batch* batch, int32_t nsteps);
fcns_status fcns_batch_destroy(fcns_batch* batch);

/* Autotuner: times, on this context's own buffers and stream, the launch
 * choices that depend on the shape -- the persistent grid of the y pass, the
 * tiling of the x pass with products, and the radix order of the run-time z
 * plan (a compiled plan is kept) -- and keeps the fastest of each for later
 * calls.  Needs a state; leaves it unchanged (results of later steps stay
 * within rounding of the untuned ones).  Synchronizes the stream; may
 * reallocate the small z twiddle tables.  report (HOST, nullable) receives a
 * one-line summary of the choices. */
fcns_status fcns_autotune(fcns_ctx* ctx, char* report, int32_t report_len);

/* Choose how rk_step runs the z pass of a stage (continuation, z
 * transforms, RK combine, projection and the back transforms of the new
 * state): on = 1 one fused kernel per stage (V* and the new state pass
 * through the caches within one workgroup), 0 three kernels (the default;
 * fcns_autotune picks the faster).  The fused form applies to FP64 contexts
 * with N' <= 288 and to stages whose output buffer is not their input (both
 * stages of o = 2); other stages keep three kernels.  EINVAL if on = 1 for a
 * context it does not apply to.  Results agree to rounding. */
fcns_status fcns_set_z_fused(fcns_ctx* ctx, int32_t on);

/* Choose how rk_step runs the y and x passes of a stage (Sec. 4.2: the y
 * back transforms of v and its derivatives, the products in x, the y
 * forward transform of the nonlinear term): planes = 0 over whole arrays
 * (the default), planes > 0 slab by slab in z, that many planes at a time,
 * so that each slab's intermediate arrays are read back soon after they
 * are written (fcns_autotune picks the faster).  Results are bitwise the
 * same.  EINVAL if planes < 0 or 4 planes > 3 nz. */
fcns_status fcns_set_slab(fcns_ctx* ctx, int32_t planes);

/* Choose the layout of rk_step's (kx, y) intermediate arrays (Sec. 4.2: v
 * and its y and z derivatives between the y back transforms and the
 * products in x): on = 0 row-major (the default), 1 blocked (each group of
 * 4 kx columns stored contiguously over y, so that the y back transforms
 * write whole contiguous blocks; fcns_autotune picks the faster).  Results
 * are bitwise the same.  EINVAL if on = 1 and the x pass cannot read that
 * layout (it needs nx = 64, 128, 256 or 512 and the wave-level x kernel). */
fcns_status fcns_set_blocked(fcns_ctx* ctx, int32_t on);

/* Lines (kx columns) per workgroup tile of the y transforms: 4 (the
 * default) or 8 (whole 128-byte rows; ny = 512 only, else EINVAL);
 * fcns_autotune picks per launch kind.  Results are bitwise the same. */
fcns_status fcns_set_y_lines(fcns_ctx* ctx, int32_t lines);

/* The context's launch choices (y grid, prefetch and tile lines per launch
 * kind, x kernel variant, slab size, intermediate layout, fused z pass, z
 * radix order) as text, "key=value" pairs separated by ';', so that a tuned
 * configuration can be kept and applied again without autotuning.
 * fcns_get_choices writes it NUL-terminated into out (EINVAL if len is too
 * small); fcns_set_choices applies such a text (keys may be omitted; EINVAL,
 * changing nothing, for an unknown key or a choice the context cannot take).
 * Choices change launch shapes only: results are the same to rounding. */
fcns_status fcns_get_choices(const fcns_ctx* ctx, char* out, int32_t len);
fcns_status fcns_set_choices(fcns_ctx* ctx, const char* text);

/* Same as fcns_rk_step, by replaying a HIP graph of one step.  The graph is
 * captured on the first call and again whenever dt changes or the launch
 * choices have changed since (fcns_set_z_fused, fcns_set_slab,
 * fcns_set_blocked, fcns_set_y_lines, fcns_set_choices, fcns_autotune);
 * capture synchronizes the stream and allocates the graph, replays allocate
 * nothing, which removes the per-kernel launch cost of small problems.
 * Results are bitwise those of fcns_rk_step.  Kernel timing does not cover
 * graph replays. */
fcns_status fcns_rk_graph(fcns_ctx* ctx, double dt, int32_t nsteps);

/* Physical state.  theta (nullable) for Boussinesq contexts; p (nullable)
 * needs keep_pressure and at least one step, and is returned with zero mean. */
fcns_status fcns_get_state(fcns_ctx* ctx, double* v, double* theta, double* p);

/* Continued spectral state for checkpoint / restart: field f (0..2 velocity,
 * 3 theta) as complex128 [N'][ny][nx/2+1] (interleaved re, im), continued
 * (kx, ky, kz) coefficients with unnormalized forward FFTs.  get copies the
 * state out; set replaces it (and resets the stored wall gradient to the one
 * passed in wall_grad, complex128 [2][2][ny][nx/2+1], or to 0 if NULL). */
fcns_status fcns_get_spectral(fcns_ctx* ctx, int32_t field, double* out);
fcns_status fcns_set_spectral(fcns_ctx* ctx, const double* const* fields, const double* wall_grad);
fcns_status fcns_get_wall_grad(fcns_ctx* ctx, double* out);

/* Kernel timing for tracing and roofline reports.  While enabled, every
 * kernel that rk_step launches is bracketed by HIP events recorded on the
 * context stream (small extra launch latency).  Classes: y_back_dy,
 * y_back_dz, x_nl, y_fwd, z_stageA, z_stageB, z_back. */
fcns_status fcns_set_timing(fcns_ctx* ctx, int32_t enable);
/* The same for a subset: bit i of mask enables class i (in the order above;
 * 0 disables timing).  Bits beyond the last class: FCNS_EINVAL.  Fewer
 * events perturb the step less. */
fcns_status fcns_set_timing_mask(fcns_ctx* ctx, int32_t mask);
fcns_status fcns_timing_reset(fcns_ctx* ctx);
/* Synchronizes the stream, then fills up to max classes: names (HOST,
 * 32 chars each, NUL-terminated), counts (HOST, launches) and ms (HOST,
 * summed event durations since the last reset); *n = classes written. */
fcns_status fcns_timing_report(fcns_ctx* ctx, int32_t max, int32_t* n, char* names,
                               int64_t* counts, double* ms);

/* Flow diagnostics of the current state (synchronizes the stream).  out
 * (HOST) receives up to nout of FCNS_NDIAG values, in this order:
 *   0 kinetic energy, one half of the grid mean of |v|^2
 *   1 grid mean of (div v)^2, the FC divergence (Sec. 6)
 *   2, 3 wall means of u^2 + v^2 (slip) at z = 0 and z = Lz
 *   4, 5 wall means of w^2 at z = 0 and z = Lz
 *   6, 7 x-y mean of du/dz at z = 0 and z = Lz
 *   8, 9 friction Reynolds number sqrt(nu |dU/dz|) (Lz/2) / nu at each wall
 *   10, 11 Nusselt number 1 - (1/gamma) <d theta/dz>_xy at each wall
 *         (Sec. 7; NaN without theta)
 *   12 grid mean of theta^2 (0 without theta)
 * Grid means are over the nx*ny*nz points; z derivatives are those of the
 * continued state (B_z(i k~z V^)). */
#define FCNS_NDIAG 13
fcns_status fcns_diagnostics(fcns_ctx* ctx, double* out, int32_t nout);

/* 1D spectra of field (0..2 velocity, 3 theta) at height index z (Sec. 6):
 * ex[kx] (HOST, nx/2+1) = sum over ky of |q^(kx, ky)|^2 with the -kx half
 * folded in, ey[ky] (HOST, ny, FFT order) = sum over all kx, both with q^
 * normalised by nx ny so that each sums to the x-y mean of q^2 at z.
 * Synchronizes the stream. */
fcns_status fcns_spectra(fcns_ctx* ctx, int32_t field, int32_t z, double* ex, double* ey);

/* Sizes of the context: N' = nz + C. */
int32_t fcns_npr(const fcns_ctx* ctx);

/* Device bytes a context for this problem allocates (state, scratch and
 * tables), without creating it.  HOST problem pointer. */
fcns_status fcns_footprint(const fcns_problem* prob, int64_t* bytes);

/* Replace the physical parameters of an existing context (viscosity,
 * diffusivity, buoyancy rate, body force) so that a resident context can serve
 * another problem of the same shape; takes effect for work enqueued after the
 * call.  EINVAL for negative nu or kappa or non-finite values. */
fcns_status fcns_set_params(fcns_ctx* ctx, double nu, double kappa, double gamma,
                            double forcing_x);

/* The hipStream_t the context enqueues on. */
void* fcns_stream(const fcns_ctx* ctx);

/* ------------------------------------------------------------------ serving
 * A request loop over independent solves of different shapes (the batched
 * serving of parameter sweeps).  A request is (problem, initial state,
 * dt, nsteps).  Requests are admitted in arrival order, first fit, while
 * fewer than max_active run and their device footprint (fcns_footprint plus
 * a staging copy of the physical fields) fits in max_bytes together with the
 * resident contexts; finished contexts stay resident and serve later
 * requests of the same shape (fcns_set_params), idle ones are evicted least
 * recently used when memory is needed.  Each context has its own
 * non-blocking HIP stream, so admitted requests overlap on the device, and
 * each request's result is the one a single-problem rk_step gives.  Steps
 * are enqueued a few at a time as earlier ones complete, and each step's
 * non-finite flag is read as it completes: a request whose state blows up
 * stops there and finishes with FCNS_ENONFINITE (its outputs not written),
 * without affecting the others.  All calls from one host thread; progress
 * happens only inside fcns_server_poll. */
typedef struct fcns_server fcns_server;

fcns_status fcns_server_create(int32_t max_active, int64_t max_bytes, fcns_server** out);
/* Launch choices for one shape (the text of fcns_get_choices, e.g. from a
 * context of that shape tuned beforehand with fcns_autotune): every context
 * the server creates afterwards for a problem of this shape (grid, box, FC
 * parameters and table, order, precision, filter) takes them.  HOST
 * pointers; the text is copied.  A context that cannot take them fails the
 * request that needed it. */
fcns_status fcns_server_set_choices(fcns_server* srv, const fcns_problem* prob,
                                    const char* choices);
/* Size-aware admission: at most max_large running requests with at least
 * large_points grid points (nx ny nz) each; while that many run, a waiting
 * large request keeps its place in the queue and smaller requests behind it
 * are admitted (small solves fill the device around large ones instead of
 * large ones sharing it).  max_large = 0 (the default): arrival order only.
 * EINVAL for max_large < 0, or max_large > 0 with large_points < 1. */
fcns_status fcns_server_set_mix(fcns_server* srv, int32_t max_large, int64_t large_points);
/* HOST pointers.  The problem (and its fc_table) is copied.  v0
 * [3][nz][ny][nx] and theta0 [nz][ny][nx] (Boussinesq) are read when the
 * request is admitted, v_out and theta_out (same shapes) are written when it
 * finishes: the caller keeps all four valid and v0, theta0 unchanged until
 * then.  *id identifies the request. */
fcns_status fcns_server_submit(fcns_server* srv, const fcns_problem* prob, const double* v0,
                               const double* theta0, double dt, int32_t nsteps, double* v_out,
                               double* theta_out, int64_t* id);
/* Progress: collect finished requests, admit queued ones.  Outputs (nullable)
 * are the queue length, the number running and the number finished so far. */
fcns_status fcns_server_poll(fcns_server* srv, int32_t* n_queued, int32_t* n_active,
                             int64_t* n_done);
/* Seconds on the server's clock (steady, from fcns_server_create). */
double fcns_server_now(const fcns_server* srv);
/* Status of a finished request (its state is then in v_out, theta_out);
 * stats (HOST, nullable, 6 doubles): submit, admit and done times (server
 * clock, s), mean, median and max step time (ms, HIP events on its stream).
 * ESTATE if not finished; ENONFINITE if the state blew up; ECANCELED if
 * cancelled. */
fcns_status fcns_server_result(fcns_server* srv, int64_t id, double* stats);
/* Per-step times (ms) of a finished request: up to max into ms (HOST). */
fcns_status fcns_server_step_times(fcns_server* srv, int64_t id, int32_t max, float* ms,
                                   int32_t* n);
/* Cancel a request: a queued one finishes at once, a running one after the
 * steps already on the device (no more are enqueued); either way its result
 * is FCNS_ECANCELED and v_out, theta_out are not written.  Other requests
 * are unaffected.  EINVAL for an unknown id; FCNS_OK (no effect) when the
 * request has already finished. */
fcns_status fcns_server_cancel(fcns_server* srv, int64_t id);
/* Forget a finished request. */
fcns_status fcns_server_release(fcns_server* srv, int64_t id);
/* Synchronize and free every context. */
fcns_status fcns_server_destroy(fcns_server* srv);
const char* fcns_server_last_error(const fcns_server* srv);

/* Message for the last error on this context (or on creation when ctx is
 * NULL). */
const char* fcns_last_error(const fcns_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FCNS_H */
