/*
 * poisson.h - C ABI of the MI355X (gfx950) direct Poisson solver.
 *
 * The library solves the second-order finite-difference Poisson equation on a
 * staggered (cell-centred) Cartesian grid by eigenfunction expansion
 * (P. Costa, "A FFT-based finite-difference solver for massively-parallel
 * direct numerical simulations of turbulent flows", Sec. 2.1):
 *
 *   sum over the three axes of the central second difference of Phi  = f
 *   (Eq. (poi); the third axis may be non-uniform, Sec. 2.1 footnote),
 *
 * with homogeneous periodic / staggered Neumann / staggered Dirichlet
 * boundary conditions (Table 1).  Two axes are diagonalised by real-to-real
 * transforms (Table 2: DFT, DCT-II/III, DST-II/III, DCT-IV, and DST-IV for the
 * Dirichlet-Neumann pair), the reduced tridiagonal systems (Eq. (poi_reduced))
 * are solved by Gauss elimination along the third axis (cyclic when that axis
 * is periodic, Sec. 3), and the backward transforms return Phi.
 *
 * Around the solve (Sec. 2): Helmholtz plans (A + shift) Phi = f with the
 * non-staggered DST-I / DCT-I pairs of an implicit diffusion step; the
 * pressure-correction steps on the staggered grid (right-hand side of
 * Eq. (poi_ns), the velocity and pressure updates); and one low-storage
 * three-substep Runge-Kutta time step of the Navier-Stokes equations on a
 * tri-periodic grid (Eq. (up)).
 *
 * Data layout: a field is nx*ny*nz values, index i + nx*(j + ny*k), x fastest.
 * All field pointers are DEVICE pointers; all other pointers are HOST pointers.
 * Streams are hipStream_t values (NULL = the legacy default stream).
 *
 * Alignment: a field the solve kernels work on must be 16-byte aligned (they
 * move neighbouring points with 16-byte accesses).  hipMalloc and torch
 * allocations are; a view at an odd element offset is not.  This covers
 * the field of solve, solve_refined_noalloc, transform_stage, tridiag_stage,
 * batch_solve, batch_bind and server_submit, phi of pressure_correction and
 * rk3_substep, phi and scratch of rk3_step, and the scratch of
 * plan_autotune.  A misaligned one is refused with POISSON_EINVAL before any
 * work is enqueued.
 *
 * Error handling: functions return POISSON_OK (0) or a negative code;
 * plan_create returns NULL on error.  The code and a message of the last
 * failing call on the calling thread are available from last_error() and
 * last_error_message().  Launch functions only enqueue work: they report
 * argument and launch errors, not results; results are valid once the stream
 * has completed.
 *
 * Thread safety: all functions may be called from several host threads.  A
 * plan owns a workspace, so one plan must not be used by two streams at once.
 */
#ifndef POISSON_H
#define POISSON_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary pair of one axis: first letter = low face (index 0), second letter
 * = high face (index n-1).  P = periodic, N = staggered Neumann (zero normal
 * gradient), D = staggered Dirichlet (zero value at the face).  Table 1 lists
 * P-P, N-N, D-D and N-D; D-N is its mirror image. */
enum poisson_bc {
  BC_PERIODIC = 0,
  BC_NN = 1,
  BC_DD = 2,
  BC_ND = 3,
  BC_DN = 4,
  /* Non-staggered (node) pairs, for the Helmholtz equations of an implicit
   * diffusion step (Sec. 2; Sec. 2.1 notes they need non-staggered
   * transforms): the n unknowns of the axis sit on grid nodes, spaced
   * uniformly by the axis spacing.  BC_DD_NODE: zero on the two boundary
   * nodes just beyond the ends (DST-I); BC_NN_NODE: the end nodes have a
   * mirrored neighbour, x_{-1} = x_1 (DCT-I).  Along z they need a uniform
   * dz.  A problem that would be singular (no Dirichlet face, no shift)
   * with a node pair is refused. */
  BC_DD_NODE = 5,
  BC_NN_NODE = 6
};

enum poisson_status {
  POISSON_OK = 0,
  POISSON_EINVAL = -1,        /* bad argument: null pointer, size < 1, bad bc, non-finite or non-positive spacing */
  POISSON_EUNSUPPORTED = -2,  /* valid problem the kernels do not handle (see plan_create) */
  POISSON_ENOMEM = -3,        /* device allocation failed */
  POISSON_EHIP = -4,          /* a HIP runtime call or kernel launch failed */
  POISSON_ENOTCONVERGED = -5  /* refinement stopped before reaching its tolerance (solve_status) */
};

enum poisson_precision {
  POISSON_FP64 = 0,           /* plain FP64 transforms and elimination */
  POISSON_FP32_REFINED = 1    /* FP32 transforms and elimination, FP64 residual/update (iterative refinement) */
};

typedef struct poisson_plan poisson_plan;

/* Build a plan for an nx x ny x nz grid (Sec. 2.1, Tables 1 and 2).
 *   dx, dy : uniform spacings of x and y (> 0, finite).
 *   dz     : HOST array of nz cell widths along z (> 0, finite); copied.  z may
 *            be non-uniform; a non-uniform z always becomes the elimination axis.
 *   bc_x, bc_y, bc_z : enum poisson_bc.
 * Axis roles: the elimination axis s is z if z is non-uniform or not periodic;
 * otherwise the first non-periodic axis among x, y; if all three are periodic,
 * x (cyclic, contiguous lines) when y and z both have supported transform
 * lengths, else z (cyclic).  The other two axes are transformed.
 * Supported sizes: every transformed axis needs an even n >= 2 whose half has
 * no prime factor above 5 and n <= 1024; the elimination axis needs
 * 1 <= n <= 512 (n >= 3 if it is periodic).  Otherwise POISSON_EUNSUPPORTED.
 * Allocates the device tables (O(nx+ny+nz) doubles) on the current device.
 * Returns NULL on error (see last_error()). */
poisson_plan* plan_create(int nx, int ny, int nz, double dx, double dy, const double* dz,
                          int bc_x, int bc_y, int bc_z);

/* Plan for the Helmholtz equation (A + shift) Phi = f, A the operator of
 * plan_create: the equations of an implicit (Crank-Nicolson) diffusion step
 * of Sec. 2, shift = -2 / (nu dt) for one velocity component.  shift <= 0
 * (finite); shift = 0 is plan_create.  Transformed axes of a node pair run
 * the DST-I / DCT-I through a real FFT of length 2(n+1) / 2(n-1), whose
 * half must have no prime factor above 5 (and be at most 512).  Everything
 * else as plan_create, including solve(), the FP32 + refinement mode and
 * the stage entry points; batches and the projection steps take staggered
 * pairs only. */
poisson_plan* plan_create_helmholtz(int nx, int ny, int nz, double dx, double dy, const double* dz,
                                    int bc_x, int bc_y, int bc_z, double shift);

/* Solve in place.  rhs: DEVICE pointer to nx*ny*nz doubles (x fastest), on the
 * plan's device, overwritten with Phi.  When no face is Dirichlet the operator
 * is singular: the solver removes the volume-weighted mean of f and returns
 * the solution with zero volume-weighted mean (this is not an error).
 * Enqueues on `stream` and returns; `rhs` must stay valid until the stream
 * completes.  FP32_REFINED plans also use their workspace. */
int solve(poisson_plan* plan, double* rhs, hipStream_t stream);

/* Release the plan and its device memory (NULL is a no-op).  Work already
 * enqueued with the plan must have completed. */
void plan_destroy(poisson_plan* plan);

/* Code and message of the last failing call on this thread (0 / "" if none).
 * The message is in thread-local storage, valid until the next failing call. */
int last_error(void);
const char* last_error_message(void);

/* Select the arithmetic of solve().  mode = POISSON_FP64 (default) or
 * POISSON_FP32_REFINED: transforms and elimination in FP32, then up to
 * max_iters refinement sweeps r = f - A Phi (FP64 seven-point residual),
 * e = FP32 solve of r, Phi += e (FP64), stopping once the error left after
 * the update, estimated from the sweep's contraction rho (the ratio of
 * successive relative updates ||e||_2 / ||Phi||_2, measured on the device)
 * as (||e||/||Phi||) rho / (1 - rho), is below tol / 10.  tol > 0,
 * 1 <= max_iters <= 64.  Allocates the refinement workspace (FP64 copy of f,
 * FP32 correction field) on first use.  Not to be called while a solve with
 * this plan is in flight. */
int plan_set_precision(poisson_plan* plan, int mode, double tol, int max_iters);

/* Device bytes the plan holds (tables + workspace), plus the bytes one solve
 * needs beyond the caller's field.  For admission by HBM footprint. */
size_t plan_workspace_bytes(const poisson_plan* plan);

/* After the stream of the last solve() has completed: number of FP32 solves
 * performed (1 + refinement sweeps; 1 for FP64 plans) and the last relative
 * update ||e||/||Phi||  (0 for FP64 plans).  Returns POISSON_ENOTCONVERGED if
 * the last refined solve stopped at max_iters above its tolerance. */
int solve_status(poisson_plan* plan, int* iters, double* last_update_rel);

/* Solve `count` independent problems, plans[i] applied in place to rhs[i]
 * (DEVICE pointers), on `stream`.  An FP32 + refinement plan may appear only
 * once (its workspace is per plan; POISSON_EINVAL otherwise).  Same result
 * per instance as solve() with the same kernel variants, bit for bit
 * (batched launches use transform variants 0-3; against solve() with the
 * staging transforms, variants 4-6, results agree to rounding).  When every
 * plan's lengths have size-specialised kernels (batch_create) and all plans
 * have one precision mode, the solves run as batched launches (see below)
 * and the call waits for `stream` to complete (it frees its temporary job
 * tables); otherwise the instances are solved one after another with
 * solve() and the call returns at once. */
int batch_solve(poisson_plan* const* plans, double* const* rhs, int count, hipStream_t stream);

/* ---- batched launches (many uneven instances, Sec. 2.1 per instance) ----
 *
 * A batch runs the three steps of Sec. 2.1 for many independent problems as
 * five launches, one per pipeline step (forward t1, forward t2, elimination,
 * backward t2, backward t1).  Each launch is a persistent grid whose work
 * items are the tiles of every instance's stage, so instances of different
 * sizes, boundary pairs and axis roles share one launch.  A batch of FP32 +
 * refinement plans runs each FP32 solve of the refinement that way, with
 * the FP64 refinement kernels of every instance (residual, update,
 * convergence test) between them; an instance whose refinement has
 * converged, or reached its max_iters, drops out of the later launches. */
typedef struct poisson_batch poisson_batch;

/* Batch over `count` plans (HOST array of plan handles, all created on the
 * current device, all FP64 or all FP32 + refinement; a refined plan at most
 * once).  The plans are borrowed: they must outlive the batch, and their
 * precision mode must not change while it exists.
 * Every transformed length must be 2M with M in {16, 32, 48, 64, 96, 128,
 * 192, 256} and every elimination length one of {64, 96, 128, 192, 256, 384,
 * 512} (POISSON_EUNSUPPORTED otherwise).  Allocates the device job tables.
 * Returns NULL on error (last_error()). */
poisson_batch* batch_create(poisson_plan* const* plans, int count);

/* Set the fields: rhs is a HOST array of `count` DEVICE pointers, rhs[i] is
 * solved in place with plans[i] (nx*ny*nz doubles, x fastest).  Copies the job
 * tables to the device synchronously; must not be called while a launch of
 * this batch may still be running.  A captured graph stays valid for an
 * FP64 batch (a refined batch captures again at its next graph launch). */
int batch_bind(poisson_batch* batch, double* const* rhs);

/* Enqueue the batched solve on `stream` (asynchronous): the five stage
 * launches, or for a refined batch the whole refinement sequence (after the
 * stream completes, solve_status() of each plan reports its refinement).
 * use_graph != 0: the first call captures the launches into a HIP graph on
 * a private stream, and every call launches that graph on `stream`. */
int batch_launch(poisson_batch* batch, hipStream_t stream, int use_graph);

/* Free the job tables and the graph.  The caller makes sure no launch of the
 * batch is still running. */
void batch_destroy(poisson_batch* batch);

/* Tune the bound batch as a whole: for each of the five steps, time its
 * launch (`reps` times after one warm-up) with every job in the variant of
 * the per-length table (see plan_autotune) and with every job in one
 * synchronous variant (transforms 0-3, elimination 0-1), and keep the
 * fastest for this batch.  A batched launch runs at the occupancy of its
 * largest job configuration, so the fastest variant of each instance alone
 * is not always the fastest together.  Synchronous; OVERWRITES the bound
 * fields (bind the real ones afterwards: the choice is kept across binds).
 * The results stay equal, bit for bit, to single solves with the chosen
 * variants.  report (HOST, may be NULL): 5 x 5 doubles, per step (forward
 * t1, forward t2, elimination, backward t2, backward t1) the average ms of
 * the table choice and of variants 0-3, -1 where a variant does not apply. */
int batch_autotune(poisson_batch* batch, int reps, hipStream_t stream, double* report);

/* ---- autotuner: kernel variants per length ----
 *
 * Each specialised length has several compiled variants: for the
 * transforms, variants 0-3 are two tile shapes (lines per tile x threads per
 * line) times two FFT radix orders (radix 8 first or radix 4 first), and
 * variants 4 and 5 (lengths 256 and 512 only; the two tile shapes) read the
 * next tile straight into LDS while the current one is transformed, and
 * variant 6 does so in FP32 for length 512 with 32 lines per tile (in FP64
 * it runs variant 0); variant 7 (FP64 length 512 on a strided axis with
 * nx >= 32; elsewhere it runs variant 4) uses 32-line tiles too, with the
 * next tile read into registers instead; for the elimination, variants 0-1
 * are two chunkings (rows per chunk x chunks per line), variant 2 reads
 * the next tile into LDS while the current one is eliminated, and variant 3
 * (contiguous lines only, elsewhere variant 0) keeps each chunk in
 * registers from its read to its write, with no tile in LDS.  All give the same result up to
 * rounding.  The variant used for a length is chosen per device, precision
 * and layout (strided: the axis is y or z; contiguous: x) from a
 * process-wide table; where nothing was tuned, a staging transform for
 * lengths 256 and 512 (variant 5 for FP64 length 256 and for FP32 length 512
 * on the contiguous axis, 6 for FP32 length 512 on the strided axes, 7 for
 * FP64 length 512 on the strided axes, else 4)
 * and variant 0 otherwise; eliminations variant 3 on contiguous lines,
 * variant 1 on strided lines of 384 points and FP32 lines of 256, else 0.  Plans and batches read the
 * table when they launch (batches when they are bound; batches use the
 * synchronous variants only: transforms 0-3, elimination 0-1). */

/* Time every variant of this plan's kernels (both transformed axes and the
 * elimination, FP64 and FP32) on `scratch` (DEVICE, at least nx*ny*nz
 * doubles; overwritten), `reps` launches each after one warm-up, and record
 * the fastest in the table.  Synchronous (waits for `stream`).  report (HOST,
 * may be NULL): 2 x (8 + 8 + 4) doubles, per precision (FP64 first) the
 * average ms of variants 0-7 of t1, 0-7 of t2 (forward + backward pair) and
 * 0-3 of the elimination, -1 where a variant does not apply. */
int plan_autotune(poisson_plan* plan, double* scratch, int reps, hipStream_t stream, double* report);

/* Variant in the table for kernel family 0 (transform) or 1 (elimination),
 * line length n, layout 0 (strided) or 1 (contiguous), fp64 1 or 0. */
int tuned_variant(int family, int n, int layout, int fp64);

/* Set that entry by hand (POISSON_EUNSUPPORTED if n has no variants). */
int set_tuned_variant(int family, int n, int layout, int fp64, int variant);

/* ---- continuous-batching server (many independent solves, Sec. 2.1 each) ----
 *
 * A server owns `slots` HIP streams and a worker thread.  Requests are queued
 * in arrival order; the request at the head is admitted as soon as a slot is
 * free and its HBM fits the budget next to what is already held, and its
 * solve is enqueued on that slot's stream at once, so it overlaps on the
 * device with the solves in flight.  HBM counted against the budget: the
 * fields of the admitted requests (8 B per point) and everything the server
 * holds on the device (refinement workspaces of the slots, 12 B per point of
 * the largest refined request a slot has run plus a status block; cached
 * plans' tables; memory waiting to be freed).  This stays within the budget
 * whenever more than one request runs; a request that fits alone is admitted
 * once the device is idle.  The server frees device memory (grown-out
 * workspaces, evicted plans) only when no request is in flight, since a free
 * waits for the whole device.  Plans are cached by problem geometry and
 * shared by concurrent requests, FP64 and refined alike (a refined solve
 * runs on its slot's workspace).  Each result equals solve() of the same
 * request on its own. */
typedef struct poisson_server poisson_server;

typedef struct poisson_request_info {
  int status;               /* POISSON_OK, POISSON_ENOTCONVERGED or an error code */
  int iters;                /* FP32 solves performed (1 for FP64) */
  int plan_cached;          /* 1 if the request reused a cached plan */
  double last_update_rel;   /* last relative refinement update (0 for FP64) */
  double submit_s;          /* host steady-clock times (seconds): submission, */
  double start_s;           /*   admission (launch enqueued), */
  double done_s;            /*   completion observed */
  long long points;         /* nx * ny * nz */
} poisson_request_info;

/* slots: streams (1..64); hbm_budget: bytes (0 = 80 % of the device's free
 * memory now); max_plans: plans kept in the cache (least recently used idle
 * plans evicted beyond it).  Uses the current device.  NULL on error. */
poisson_server* server_create(int slots, size_t hbm_budget, int max_plans);

/* Queue one solve (arguments as plan_create, plus precision mode, tolerance and
 * sweep limit as plan_set_precision; field: DEVICE pointer, nx*ny*nz doubles,
 * solved in place, owned by the caller and kept alive until server_wait
 * returns for this request).  producer: the stream on which the caller
 * wrote the field (NULL = the legacy default stream); the solve runs after
 * the work enqueued on it before this call.  dz is copied.  Returns a request
 * id >= 0, or a negative error code (POISSON_EUNSUPPORTED if the request
 * alone, field and refinement workspace, exceeds the budget). */
long long server_submit(poisson_server* server, int nx, int ny, int nz, double dx, double dy,
                        const double* dz, int bc_x, int bc_y, int bc_z, int precision,
                        double tol, int max_iters, double* field, hipStream_t producer);

/* Block until request `id` has completed; fills *info (may be NULL) and
 * forgets the request.  Returns its status. */
int server_wait(poisson_server* server, long long id, poisson_request_info* info);

/* Plan-cache counters, plans resident (cached, and evicted ones not yet
 * freed) and the admission budget in bytes (any pointer may be NULL). */
int server_stats(poisson_server* server, long long* plan_hits, long long* plan_misses,
                 int* plans_resident, size_t* budget);

/* Device bytes the server holds now (workspaces, plan tables, memory
 * waiting to be freed) and the largest total of held bytes plus admitted
 * fields seen at an admission (any pointer may be NULL). */
int server_usage(poisson_server* server, size_t* held_bytes, size_t* peak_bytes);

/* Finish every queued request, stop the worker, free the cached plans. */
void server_destroy(poisson_server* server);

/* ---- the pressure-correction steps around the solve (Sec. 2) ----
 *
 * The substep of the paper's projection method: the right-hand side
 * div(u*) / (gamma_k dt) of Eq. (poi_ns), the solve, and the updates
 * u = u* - gamma_k dt grad(Phi), p = p + Phi, on the staggered grid of the
 * plan (its widths and boundary pairs; the boundary pair of Phi along an
 * axis sets that of the normal velocity: P periodic, N an impermeable
 * wall whose velocity the projection leaves as it is, D an open face with
 * Phi = 0 on it).
 *
 * Layout (DEVICE arrays of doubles, x fastest): Phi, p and rhs at the
 * cells, nx*ny*nz.  The velocity component along an axis on the faces
 * normal to it: along a periodic axis of n cells n faces, face f between
 * cells f-1 (cyclically) and f; along a walled axis n + 1 faces, face 0
 * the low wall and face n the high wall.  So u is (nx + wx) x ny x nz, v
 * nx x (ny + wy) x nz, w nx x ny x (nz + wz), with w_ = 1 on a walled axis.
 * Face gradients use centre distances (the mean of the two widths) and,
 * at a wall, the ghost rule of the solve (Neumann: zero gradient;
 * Dirichlet: 2 Phi_edge / h_edge inward), so that the divergence of the
 * gradient is the solve's operator and the projected velocity is
 * divergence-free up to rounding.  When the operator is singular (no
 * Dirichlet face) only a prediction whose net flux through the walls is
 * zero can be made divergence-free; the solve removes the mean of the
 * right-hand side as usual. */

/* rhs = div(u, v, w) / gamma_dt at every cell (gamma_dt finite, non-zero).
 * Enqueued on `stream`. */
int projection_rhs(poisson_plan* plan, const double* u, const double* v, const double* w,
                   double gamma_dt, double* rhs, hipStream_t stream);

/* In place: u, v, w -= gamma_dt * grad(phi) on every face, p += phi at every
 * cell.  Enqueued on `stream`. */
int projection_update(poisson_plan* plan, const double* phi, double gamma_dt, double* u,
                      double* v, double* w, double* p, hipStream_t stream);

/* The whole step on `stream`: projection_rhs into phi (caller-owned, DEVICE,
 * nx*ny*nz doubles), solve(plan, phi) in the plan's precision mode, then
 * projection_update.  On return phi holds the correction pressure. */
int pressure_correction(poisson_plan* plan, double* u, double* v, double* w, double* p,
                        double gamma_dt, double* phi, hipStream_t stream);

/* ---- one Navier-Stokes time step (Sec. 2, Eq. (up) and the pressure
 * correction of every substep) ----
 *
 * The low-storage three-substep Runge-Kutta scheme with alpha = {8/15,
 * 5/12, 3/4}, beta = {0, -17/60, -5/12}, gamma = alpha + beta, on a plan
 * periodic along every axis with uniform widths (the Taylor-Green case of
 * Sec. 4.1); other plans give POISSON_EUNSUPPORTED.
 *
 * Fields (all DEVICE, caller-owned, x fastest, N = nx*ny*nz doubles each):
 *   vel   3 N: u, v, w one after another; component c at (i, j, k) lives on
 *         the low face of cell (i, j, k) normal to axis c.  In / out.
 *   work  3 N: the prediction u* (scratch; overwritten).
 *   ad    6 N: two buffers of AD = -(u . grad) u + nu lap(u) (advection in
 *         divergence form, second-order central differences), each 3 N:
 *         substep 1 writes its AD into the first, substep 2 reads the first
 *         and writes its own into the second, substep 3 reads the second and
 *         writes nothing (the next step's first substep needs no AD).
 *   p     N: the pressure p^{k-1/2} at cell centres; gains phi.  In / out.
 *   phi   N: the correction pressure of the substep (zero mean).  Out.
 * Arrays must not overlap.  Enqueued on `stream`; the solve uses the plan's
 * precision mode.  dt > 0, nu >= 0 (POISSON_EINVAL otherwise). */

/* The prediction of substep k (1, 2, 3) and the right-hand side of its
 * pressure equation (Eq. (up), Eq. (poi_ns)): work = u* = u + dt (alpha_k AD
 * + beta_k AD_prev - gamma_k grad p), ad as described above, and
 * rhs (N doubles) = div(u*) / (gamma_k dt).  vel and p are only read. */
int rk3_predict(poisson_plan* plan, int k, double dt, double nu, const double* vel, double* work,
                double* ad, const double* p, double* rhs, hipStream_t stream);

/* Substep k (1, 2, 3): rk3_predict into work and phi, phi = solve(phi),
 * u = u* - gamma_k dt grad phi, p += phi. */
int rk3_substep(poisson_plan* plan, int k, double dt, double nu, double* vel, double* work,
                double* ad, double* p, double* phi, hipStream_t stream);

/* One time step: substeps 1, 2, 3 (gamma_1 + gamma_2 + gamma_3 = 1), with
 * the same results as rk3_substep three times up to rounding.  The
 * projection of substeps 1 and 2 is applied by the next substep's
 * prediction as it reads its input instead of in a sweep of its own;
 * scratch (DEVICE, 2 N doubles, overwritten) holds the intermediate
 * pressure and correction pressure.  On return vel and p hold the new
 * velocity and pressure, phi the third substep's correction pressure. */
int rk3_step(poisson_plan* plan, double dt, double nu, double* vel, double* work, double* ad,
             double* p, double* phi, double* scratch, hipStream_t stream);

/* ---- refined solve that allocates nothing ----
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * FP32 + FP64 refinement as solve() on a POISSON_FP32_REFINED plan (same
 * kernels, same launch sequence: the same bits), whatever the plan's own
 * precision mode, but its workspace (FP64 copy of f, FP32 residual /
 * correction field, status block) is a static array of the library, 256 MiB
 * per device, held from the library's load on that device until the
 * process ends.  The call allocates nothing and calls no allocating
 * routine.  Every call on a device uses that device's one array and leaves
 * its contents behind (each call re-initialises what it reads): calls that
 * overlap on one device, on any streams, race and give wrong results; the
 * caller orders them (one stream, or events). */

/* Largest nx*ny*nz that solve_refined_noalloc accepts (the workspace takes
 * 12 B per point plus a status block). */
size_t refined_noalloc_max_points(void);

/* Refined solve of rhs in place (DEVICE, nx*ny*nz doubles, x fastest) with
 * tolerance tol (> 0) and at most max_iters FP32 solves (1..64), as
 * plan_set_precision describes, on the workspace above, enqueued on
 * `stream`.  status_out (DEVICE, 3 doubles, may be NULL) receives at the end
 * of the stream: FP32 solves performed, 1.0 if the tolerance was reached
 * (else 0.0), and the last relative update.  solve_status() does not report
 * this call.  POISSON_EUNSUPPORTED if the grid has more than
 * refined_noalloc_max_points() points; POISSON_EINVAL for bad arguments or
 * when the current device is not the plan's. */
int solve_refined_noalloc(poisson_plan* plan, double* rhs, double tol, int max_iters,
                          double* status_out, hipStream_t stream);

/* ---- stage entry points (the steps of Sec. 2.1, for stage-level checks) ---- */

/* Axis roles chosen by the plan: roles[0] = t1, roles[1] = t2 (the transformed
 * axes, forward order), roles[2] = s (elimination axis); 0 = x, 1 = y, 2 = z. */
int plan_roles(const poisson_plan* plan, int roles[3]);

/* Step 1 / 3 for one transformed axis (role 0 = t1, 1 = t2), in place on an
 * FP64 DEVICE field: inverse = 0 applies the forward transform of Table 2
 * (unnormalised, DFT in Table 2's interleaved order), inverse = 1 the backward
 * operator of Table 1 ((1/n) IDFT, (1/2n) DCT-III, (1/2n) DST-III, (1/2n) DCT-IV,
 * (1/2n) DST-IV). */
int transform_stage(poisson_plan* plan, int role, int inverse, double* field, hipStream_t stream);

/* Step 2: solve the reduced tridiagonal systems (Eq. (poi_reduced)) of every
 * column along s, in place on an FP64 DEVICE field holding the transformed
 * right-hand side in the storage order of transform_stage.  The column of
 * wavenumber zero of a singular problem is projected, pinned and gauged to
 * zero weighted mean. */
int tridiag_stage(poisson_plan* plan, double* field, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* POISSON_H */
