/*
 * hjw.h - C ABI of the MI355X WENO-L Hamilton-Jacobi library.
 *
 * Solves phi_t + H(x, t, phi, D phi) = 0, phi(x,0) = phi0(x), on a uniform 1-D or 2-D
 * grid (Rathan & Biswas, arXiv:1909.13263, eq. (1.1) restricted to built-in Hamiltonian
 * families, see hjw_ham) with the fifth-order arc-length WENO derivatives of
 * Section 2 (Steps 1-4), the Lax-Friedrichs numerical Hamiltonian (eq. LF) and
 * third-order TVD Runge-Kutta in time (Step 5); two dimensions are handled
 * dimension by dimension (the Note closing Section 2).
 *
 * Conventions shared by every entry point
 *   - Every call returns an hjw_status; nothing throws or aborts across the ABI.
 *     hjw_last_error() returns a thread-local message for the last failure.
 *   - Arrays are row-major with x fastest: phi[j*nx + i] = phi(x_i, y_j).  phi is
 *     exchanged as FP64 in every precision mode.
 *   - A periodic or Dirichlet axis of n points covers [lo, hi) with x_i = lo + i*h,
 *     h = (hi-lo)/n; an extrapolated axis is cell-centred, x_i = lo + (i+1/2)*h.
 *     n >= 8 per axis (see hjw_bc).
 *   - The library owns hjw_grid objects.  The caller owns every pointer it passes:
 *     host arrays, device arrays and the device workspace given to hjw_bind, which
 *     must stay allocated until hjw_grid_destroy.
 *   - One grid is not thread-safe; distinct grids may be used from distinct threads.
 *   - After a non-finite value is detected a grid is failed: every call except
 *     hjw_set_phi, hjw_get_info and hjw_grid_destroy returns HJW_ESTATE.
 */
#ifndef HJW_H
#define HJW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HJW_OK = 0,
    HJW_EINVAL = -1,     /* bad argument or unsupported combination            */
    HJW_ENOMEM = -2,     /* workspace too small / host allocation failed        */
    HJW_EHIP = -3,       /* a HIP runtime call failed (message has the code)     */
    HJW_ESTATE = -4,     /* call not valid in the grid's state (unbound, failed) */
    HJW_ENONFINITE = -5, /* a non-finite derivative, flux or phi appeared        */
    HJW_EBUSY = -6       /* resource in use                                      */
} hjw_status;

/* Boundary per axis:
 *   HJW_BC_PERIODIC   nodes x_i = lo + i h, h = (hi - lo)/n, wrapped;
 *   HJW_BC_EXTRAP     cell-centred nodes x_i = lo + (i + 1/2) h, three ghosts on each
 *                     side extrapolated linearly through the two end nodes;
 *   HJW_BC_DIRICHLET  nodes x_i = lo + i h; the three outermost node layers hold the
 *                     boundary data (their values in the phi given to hjw_set_phi, or
 *                     to hjw_server_submit) and are never updated; their derivatives
 *                     are left out of the dissipation ranges.  Needs n >= 7 (n >= 8
 *                     holds for every grid).  Example 3.10 of Section 3 names a
 *                     Dirichlet boundary without its data; this is the reading. */
typedef enum { HJW_BC_PERIODIC = 0, HJW_BC_EXTRAP = 1, HJW_BC_DIRICHLET = 2 } hjw_bc;

/* Arithmetic of the stencil (candidates, indicators, weights, flux):
 *   HJW_FP64        everything in FP64;
 *   HJW_FP32_MIXED  stencil in FP32 on differences taken in FP64; phi stored and
 *                   accumulated in FP64; dissipation and time step in FP64;
 *   HJW_FP32        as FP32_MIXED but phi stored in FP32 (RK combination still
 *                   evaluated in FP64 before rounding). */
typedef enum { HJW_FP64 = 0, HJW_FP32_MIXED = 1, HJW_FP32 = 2 } hjw_prec;

/* Smoothness indicators of the fifth-order reconstruction (the candidates, linear
 * weights (1, 6, 3)/10, eps = 1e-6 and the weight formula of eq. (WLOC1) are shared):
 *   HJW_WENO_L   the paper's arc-length indicators, Section 2 Step 4 (default);
 *   HJW_WENO_JP  Jiang and Peng's indicators, the scheme the paper compares with in
 *                Section 3 (Tables 1-4, right halves). */
typedef enum { HJW_WENO_L = 0, HJW_WENO_JP = 1 } hjw_scheme;

/* Built-in Hamiltonians H(u, v), u = phi_x, v = phi_y (v = 0 in 1-D):
 *   LINEAR   p[0]*u + p[1]*v                    (Example 3.1)
 *   BURGERS  (p[0]*u + p[1]*v + p[2])^2 / 2     (Examples 3.3, 3.6)
 *   NEGCOS   -cos(p[0]*u + p[1]*v + p[2])       (Examples 3.2, 3.4; 3.10 with p[2] = pi/2)
 *   NORM     p[0]*sqrt(u^2 + v^2 + p[1])        (Example 3.12 with p[1] = 1;
 *                                                level-set motion with p[1] = 0)
 *   QUARTIC  (s^2 - 1)(s^2 - 4) / 4, s = p[0]*u + p[1]*v + p[2]   (Example 3.8)
 *   CONTROL  sin(y) u + (sin(x) + sign v) v - sin(y)^2/2 - (1 - cos x), at the node
 *            (x, y); no parameters                                (Example 3.11)
 *   CURVATURE p[0]*sqrt(u^2 + v^2 + p[1]) plus the curvature term of Example 3.13 with
 *            weight eps = p[2] >= 0: the operator gains eps N / (1 + phi_x^2 + phi_y^2),
 *            N = (1 + phi_y^2) phi_xx - 2 phi_x phi_y phi_xy + (1 + phi_x^2) phi_yy, from
 *            second-order central differences over the node's 3 x 3 neighbourhood, and
 *            the time-step rate gains 2 eps (1/dx^2 + 1/dy^2).  Example 3.13 is
 *            p = {-1, 1, eps}.  2-D grids with periodic or Dirichlet axes only (EINVAL
 *            otherwise).
 *   TIMED    cos(p[2]*t) (p[0]*u + p[1]*v) + p[3]*phi: the general form of eq. (1.1),
 *            depending on the time and on the node's value (no example of the paper).
 *            The three RK stages evaluate it at t_n, t_n + dt and t_n + dt/2 with each
 *            stage's own phi; the dissipation is |p[0]|, |p[1]|, and the time-step rate
 *            gains |p[3]|.  Its grids run kernels of their own with 64 x 16 tiles
 *            (EINVAL with HJW_OPT_TILE_ROWS = 32).
 * The dissipation of eq. (LF) is the maximum of |H_u|, |H_v| over the box of the
 * step's derivative ranges (CONTROL: the bounds 1 and 2 of its coefficients). */
typedef enum {
    HJW_H_LINEAR = 0,
    HJW_H_BURGERS = 1,
    HJW_H_NEGCOS = 2,
    HJW_H_NORM = 3,
    HJW_H_QUARTIC = 4,
    HJW_H_CONTROL = 5,
    HJW_H_CURVATURE = 6,
    HJW_H_TIMED = 7
} hjw_ham;

/* Options for hjw_set_option. */
typedef enum {
    HJW_OPT_USE_GRAPH = 0,     /* 1 (default): replay captured HIP graphs of whole RK steps;
                                  0: launch every kernel eagerly.  Results are identical. */
    HJW_OPT_KERNEL_EVENTS = 1, /* 1: launch eagerly and bracket every kernel of a step with
                                  HIP events on the grid's stream; resets the totals that
                                  hjw_kernel_times reports.  0 (default): off. */
    HJW_OPT_TILE_ROWS = 2,     /* 2-D tile height: 16 (default: 64 x 16 nodes) or 32 (64 x 32
                                  nodes, 8-node segments only; not with HJW_H_TIMED, whose
                                  kernels take 16-row tiles).  Results are identical. */
    HJW_OPT_SEGMENT = 3,       /* nodes each thread marches in the 2-D sweeps: 0 (default)
                                  automatic, 4 (FP32 stencil, 16-row tiles: 512 threads per
                                  tile) or 8 (256 threads per 16-row tile).  Results are
                                  identical. */
    HJW_OPT_PLAN = 4,          /* where a 2-D step's dissipation and time step are computed:
                                  0 (default) automatic, 1 in every workgroup of the second
                                  stage, 2 in a one-wave launch of its own between the first
                                  and second stages (chosen automatically above 2048 tiles).
                                  Results are identical. */
    HJW_OPT_DISSIPATION = 5    /* alpha of eq. (LF), alpha = max |H_1|, whose range the paper
                                  leaves open: 0 (default) over the box of the step's
                                  derivative ranges, held for the step's three stages; 1 per
                                  node and stage over the node's own box [u-, u+] x [v-, v+]
                                  (local Lax-Friedrichs; the printed Table 2 follows it).  The
                                  time step keeps the global alpha.  Not with
                                  HJW_OPT_TILE_ROWS = 32 (EINVAL). */
} hjw_option;

typedef struct hjw_grid hjw_grid;

typedef struct {
    int64_t steps;    /* RK3 steps taken since the last hjw_set_phi                  */
    double t;         /* current time                                               */
    double last_dt;   /* time step of the last step                                 */
    double alpha_x;   /* dissipation of the last step, max |H_1| over the box (LF)  */
    double alpha_y;
    double range[4];  /* the box: min/max of phi_x^-, phi_x^+ and of phi_y^-, phi_y^+ */
} hjw_info;

/* Create a grid.  dim = 1 or 2; n[d], lo[d], hi[d], bc[d] per axis, x first.
 * Nothing is allocated on the device.  *out receives the grid. */
hjw_status hjw_grid_create(int dim, const int64_t *n, const double *lo, const double *hi,
                           const int *bc, int prec, hjw_grid **out);

/* Bytes of device workspace the grid needs (its whole HBM footprint: phi, the
 * stage buffer, the three stage-1 flux arrays, block partials and the step state). */
hjw_status hjw_workspace_bytes(const hjw_grid *g, size_t *bytes);

/* Bind device memory (>= hjw_workspace_bytes, 256-byte aligned) and a HIP stream
 * (hipStream_t; NULL lets the library create its own blocking stream).  The
 * workspace and stream are borrowed.  Rebinding is allowed; phi must be set again. */
hjw_status hjw_bind(hjw_grid *g, void *dev_workspace, size_t bytes, void *hip_stream);

/* Choose the Hamiltonian (see hjw_ham) and its parameters (nparams <= 4). */
hjw_status hjw_set_hamiltonian(hjw_grid *g, int kind, const double *params, int nparams);

/* Choose the smoothness indicators (hjw_scheme; HJW_WENO_L until set).  Takes effect
 * from the next step; HJW_EINVAL for an unknown scheme. */
hjw_status hjw_set_scheme(hjw_grid *g, int scheme);

/* Copy phi0 (FP64, nx*ny values, host or device memory) into the grid; t := 0,
 * steps := 0, the failed state is cleared.  Synchronous. */
hjw_status hjw_set_phi(hjw_grid *g, const double *phi0, int on_device);

/* Advance with TVD-RK3 until t = t_final or max_steps steps were taken
 * (max_steps <= 0: no limit).  dt = cfl / (alpha_x/dx + alpha_y/dy), clamped so
 * that the last step lands on t_final exactly.  Blocking; fills *info if not NULL.
 * Returns HJW_ENONFINITE (and fails the grid) if a non-finite value appears. */
hjw_status hjw_step_to(hjw_grid *g, double t_final, double cfl, int64_t max_steps,
                       hjw_info *info);

/* Copy phi (FP64, nx*ny values) out to host or device memory.  Synchronous. */
hjw_status hjw_get_phi(const hjw_grid *g, double *out, int on_device);

/* The fifth-order WENO-L one-sided derivatives of the current phi (Steps 1-4):
 * phi_x^-, phi_x^+ and, in 2-D, phi_y^-, phi_y^+ (vm, vp ignored in 1-D), written
 * as FP64 to caller-owned device arrays of nx*ny values.  Synchronous. */
hjw_status hjw_derivatives(hjw_grid *g, double *um, double *up, double *vm, double *vp);

/* Current step counters and last step's dissipation/time step. */
hjw_status hjw_get_info(const hjw_grid *g, hjw_info *info);

hjw_status hjw_set_option(hjw_grid *g, int option, int64_t value);

/* With HJW_OPT_KERNEL_EVENTS on: total milliseconds and launch counts of the
 * kernels of a step since the option was switched on, in the order
 * [0] derivatives of phi^n and range slots, [1] the plan launch (dissipation and
 * time step; none where the second stage plans for itself), [2] second stage,
 * [3] third stage.  ms[4] and count[4] are caller-owned. */
hjw_status hjw_kernel_times(const hjw_grid *g, double *ms, int64_t *count);

/* Average duration in milliseconds of each kernel of a step (ms[0] first stage,
 * ms[1] the plan launch, 0 where the second stage plans for itself, ms[2] second,
 * ms[3] third stage; ms holds 4 values, caller-owned), each launched reps times back
 * to back on the grid's stream between two HIP events, on the grid's current phi.
 * Ahead of them the GPU waits about 2 ms in a hold kernel while the host submits every
 * launch, then runs two untimed launches of the same kernel: the timed ones start back
 * to back however slowly the host submits.
 * Takes one real step first; afterwards phi is undefined and must be set again
 * (hjw_set_phi) before stepping. */
hjw_status hjw_time_kernels(hjw_grid *g, int reps, double *ms);

/* Release the grid (its graphs, events and own stream); the workspace is the
 * caller's.  NULL is ignored. */
void hjw_grid_destroy(hjw_grid *g);

/* One whole solve that allocates nothing, for callers that cannot allocate device
 * memory (no hipMalloc/hipFree: serving loops with a fixed memory budget, harnesses that
 * forbid allocation).  The same as hjw_grid_create + hjw_bind + hjw_set_hamiltonian +
 * hjw_set_phi + hjw_step_to + hjw_get_phi (WENO-L, global dissipation, 16-row tiles,
 * kernels launched without graphs), with the same results bit for bit.
 *   dim, n, lo, hi, bc, prec  as for hjw_grid_create; at most 2^20 nodes (HJW_ENOMEM
 *                             beyond that);
 *   ham, params, nparams      as for hjw_set_hamiltonian;
 *   phi                       device array of nx*ny FP64 values, caller-owned: phi0 on
 *                             entry, phi at the final time on return (in FP64 and the
 *                             FP32 stencil it is updated in place while stepping);
 *   t_final, cfl, max_steps   as for hjw_step_to; info (host, may be NULL) as there;
 *   hip_stream                hipStream_t, borrowed (NULL: the default stream).
 * The grid's stage buffer, flux records, range slots and step records (and phi in FP32
 * storage) live in a fixed device array of the library, 32 MiB + 4 KiB, of which each
 * device the library runs on keeps one copy until the process ends.  Every call on a
 * device reuses that device's copy, so calls that overlap in time on one device race.
 * Synchronous; returns HJW_ENONFINITE if phi0 or a later value is not finite. */
hjw_status hjw_solve_noalloc(int dim, const int64_t *n, const double *lo, const double *hi,
                             const int *bc, int prec, int ham, const double *params,
                             int nparams, double *phi, double t_final, double cfl,
                             int64_t max_steps, hjw_info *info, void *hip_stream);

/* ----------------------------------------------------------------------------
 * Served stream: many independent 2-D solves batched into the same launches.
 *
 * A server owns no memory: the caller gives it a device pool, from which it
 * places each admitted solve's phi, stage buffer and flux records (the footprint
 * hjw_server_footprint reports).  Requests are admitted first-in first-out as
 * soon as a slot and pool space are free; every batched step advances each
 * admitted solve by one RK3 step with its own dt, in three launches that cover
 * the tiles of all admitted solves; solves that reach t_final are retired, their
 * phi copied to host memory and their pool space released, and waiting requests
 * are admitted in their place (continuous batching).  Each solve's result is the
 * same as that of hjw_step_to on the same grid with the same precision.
 * One server is not thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct hjw_server hjw_server;

typedef struct {
    int64_t n[2];      /* nodes along x and y (>= 8 each)                        */
    double lo[2];      /* domain, as for hjw_grid_create                          */
    double hi[2];
    int bc[2];         /* hjw_bc per axis                                         */
    int ham;           /* hjw_ham                                                 */
    double params[4];  /* Hamiltonian parameters                                  */
    double t_final;    /* solve from t = 0 to t_final                             */
    double cfl;        /* CFL number, as for hjw_step_to                          */
    int scheme;        /* hjw_scheme                                              */
    int reserved;      /* 0                                                       */
} hjw_request;

typedef struct {
    int64_t submitted, queued, active, done, failed;
    int64_t batched_steps;   /* batched steps launched                         */
    double node_stages;      /* nodes x RK stages advanced, all solves        */
    size_t pool_bytes, pool_in_use, pool_peak;
} hjw_server_stats;

/* Pool bytes one request occupies while admitted (prec as in hjw_prec). */
hjw_status hjw_server_footprint(int prec, const hjw_request *req, size_t *bytes);

/* Create a server over a caller-owned device pool (256-byte aligned) for up to
 * max_active concurrent solves (1..1024); hip_stream as for hjw_bind.  The server also
 * pins host memory of its own: pinned staging for uploads and results, and an inbox for
 * queued phi0 of a quarter of the pool (at most 1 GiB; none if pinning fails). */
hjw_status hjw_server_create(int prec, void *dev_pool, size_t pool_bytes, int max_active,
                             void *hip_stream, hjw_server **out);

/* Queue a request with phi0 (FP64 host array of n[0]*n[1] values, copied before the
 * call returns: into the pinned inbox when it has room, else into host memory).
 * HJW_ENOMEM if the request could never fit the pool.  *id receives its id. */
hjw_status hjw_server_submit(hjw_server *s, const hjw_request *req, const double *phi0,
                             int64_t *id);

/* Run the stream for `chunks` chunks of batched steps and return.  The server keeps
 * two chunks queued on its stream while anything is admitted: each of the `chunks`
 * rounds waits for the oldest queued chunk to end, retires the solves it finished
 * (their phi is copied out behind the chunk still queued) and admits waiting
 * requests, so the GPU does not wait for the host between chunks.  A chunk may still
 * be running on return; the next call continues from it.  When nothing is admitted
 * on return, every queued chunk and copy has ended and every finished request is
 * reported by hjw_server_completed; returns at once when nothing is queued or
 * admitted.  *active (at most max_active) and *queued (optional) receive the counts
 * on return.  A request's finish time is when its result reached host memory. */
hjw_status hjw_server_run(hjw_server *s, int chunks, int64_t *active, int64_t *queued);

/* Ids of requests finished (done or failed) since the last call, up to cap. */
hjw_status hjw_server_completed(hjw_server *s, int64_t *ids, int cap, int *count);

/* Result of a finished request: phi (FP64 host array, may be NULL), its step
 * info, and its submit and finish times in seconds on the server's clock.
 * Returns the request's own status (HJW_OK, or HJW_ENONFINITE if it failed) and
 * releases it; HJW_ESTATE if the request is not finished. */
hjw_status hjw_server_result(hjw_server *s, int64_t id, double *phi_out, hjw_info *info,
                             double *t_submit, double *t_finish);

/* Counters of the server since creation. */
hjw_status hjw_server_get_stats(const hjw_server *s, hjw_server_stats *stats);

/* Seconds on the server's clock (the clock of t_submit / t_finish). */
double hjw_server_clock(const hjw_server *s);

/* Release the server (its graphs and own stream); queued and admitted requests are
 * dropped.  The pool is the caller's.  NULL is ignored. */
void hjw_server_destroy(hjw_server *s);

/* Thread-local description of the last error ("" if none). */
const char *hjw_last_error(void);

/* Library version string. */
const char *hjw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HJW_H */
