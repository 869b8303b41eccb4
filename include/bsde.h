/*
 * bsde.h -- C ABI of the MI355X (gfx950) library for the multistep scheme for
 * backward stochastic differential equations of Kapllani & Teng,
 * "Multistep schemes for solving backward stochastic differential equations
 * on GPU" (arXiv:1909.13560).
 *
 * The library runs the backward time sweep of the fully discrete scheme
 * (Section 2.2 eq (20), Gauss-Hermite expectations eq (21), algorithm step 3
 * of Section 3.1) on one GPU.  The problem statement follows the paper: the
 * BSDE -dy = f(t, y, z) dt - z dW with X_t = x + drift t + vol W_t (eq (1)-(2),
 * eq (33) for the log-price), the time grid N, the multistep orders K_y, K_z,
 * the truncated uniform space grid (Section 3.1 step 1), the Gauss-Hermite
 * order L and the Picard iteration (step 3).  The terminal condition g and the
 * K - 1 further initial layers (step 2) are computed by the caller on the host
 * and handed over as device arrays.
 *
 * Conventions shared by all entry points:
 *   - Every function returns a bsde_status; nothing aborts or throws across
 *     the ABI.  On an error no output is written unless stated otherwise.
 *   - Device pointers are HIP device addresses on the current device; the
 *     caller owns them.  Host pointers are plain host memory.
 *   - "stream" is a hipStream_t passed as void*; NULL is the default stream.
 *     Work is enqueued asynchronously on it; an entry point that fills a
 *     bsde_stats synchronises that stream before it returns.
 *   - Grid values are double precision in the caller's buffers for both
 *     precision modes; BSDE_FP32_COMP only changes the arithmetic inside.
 */
#ifndef BSDE_H
#define BSDE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSDE_OK = 0,
    BSDE_EINVAL = 1,       /* invalid argument or problem                         */
    BSDE_ENOMEM = 2,       /* host or device allocation failed                    */
    BSDE_EDEVICE = 3,      /* a HIP call failed (no device, launch failure, ...)  */
    BSDE_EUNSUPPORTED = 4, /* valid problem outside what the library implements  */
    BSDE_ENOCONV = 5,      /* Picard did not reach the tolerance at some point    */
    BSDE_ENONFINITE = 6,   /* a non-finite value appeared in the output layer     */
    BSDE_ESCRATCH = 7      /* plan's workspace exceeds the static workspace       */
} bsde_status;

typedef enum {
    /* f = p0 y + p1 z1 + p2 z2 + p3 (Black-Scholes, eq (29)-(30), with
     * p0 = -r, p1 = -(mu - r + delta)/sigma; the sine problem f = y/2 - z)   */
    BSDE_DRIVER_LINEAR = 0,
    /* f = -r y - theta z + s (R - r) min(y - z/sigma, 0),
     * p = {r, R, theta, sigma, s}: lending rate r, borrowing rate R          */
    BSDE_DRIVER_BIDASK = 1,
    /* Example 1, eq (22): f = -y^3 + 5/2 y^2 - 3/2 y                          */
    BSDE_DRIVER_CUBIC = 2,
    /* Example 2, eq (24): f = (e^{t^2} - 4 t y - 3 e^{t^2 - y e^{-t^2}}
     *                          + z^2 e^{-t^2}) / 2                              */
    BSDE_DRIVER_EXP = 3
} bsde_driver_kind;

/* First term of the z equation (Section 2.2).  Eq (12) holds
 * E[y_{t_{n+1}} dW_{t_{n+1}}]; the scheme of eq (20) replaces it by
 * dt E[z_{t_{n+1}}] (the relation stated below eq (12)).  The YDW form keeps
 * E[y^{n+1} dW_{n+1}] / dt instead: with K_z = 1 it is second order in z
 * (the printed form is first order there), with K_z >= 2 the multistep z
 * recurrence built on it is unstable. */
typedef enum {
    BSDE_ZFORM_EZ = 0,  /* E[z^{n+1}] (eq (20))                                  */
    BSDE_ZFORM_YDW = 1  /* E[y^{n+1} dW_{n+1}] / dt; FP64 only (the weights
                           dW/dt ~ 1/sqrt(dt) would amplify the FP32 form's
                           rounding of the stored layers)                       */
} bsde_z_form;

/* The interpolant of the layers between grid points (Section 3.3). */
typedef enum {
    BSDE_INTERP_SPLINE = 0,      /* natural cubic spline (d = 2: tensor product)    */
    BSDE_INTERP_BICUBIC_FD = 1   /* d = 2: the paper's bicubic interpolation from the
                                    values and the first and mixed derivatives,
                                    these by fourth-order finite differences
                                    (central inside, one-sided at the two points
                                    next to each end); needs n_x >= 5 per axis */
} bsde_interp;

/* How the conditional expectations of eq (20) are computed. */
typedef enum {
    BSDE_QUAD_GH = 0,    /* Gauss-Hermite quadrature of the spline, eq (21)     */
    BSDE_QUAD_EXACT = 1  /* the exact Gaussian expectation of the spline: a
                            banded Toeplitz operator on the uniform grid, applied
                            on FP64 matrix cores; no quadrature aliasing, so it
                            stays stable at stability ratios far above 16.
                            Linear driver, constant coefficients, FP64, d = 1;
                            L is not used                                        */
} bsde_quad;

typedef enum {
    BSDE_FP64 = 0,      /* all arithmetic in double precision                   */
    BSDE_FP32_COMP = 1  /* d = 1: the ring of time layers and the node
                           interpolation and driver evaluations in single
                           precision; the terms that carry the size of the
                           solution (the y-hat and z-hat expectations) summed
                           in double precision, the small f-hat terms per
                           layer in single precision and then added in double;
                           spline solve, z combination and Picard in double
                           precision.  d = 2: the ring in single precision,
                           all arithmetic in double.  Both store each new
                           value with the rounding residual of the layer it
                           came from added (error feedback) and keep the new
                           residual in the ring.  Error against the FP64
                           form: 2.8e-7 relative over the whole grid (bid-ask
                           call, 262144 points, 1024 steps)                    */
} bsde_precision;

/* One BSDE in one (d = 1) or two (d = 2, Section 5 Examples 4-5) space
 * dimensions on a uniform (tensor) grid.  Fields indexed [2] use entry 0
 * only when d = 1. */
typedef struct {
    int d;              /* space dimension, 1 or 2                               */
    double T;           /* terminal time, > 0                                    */
    int n_t;            /* N: time steps, dt = T/N, N >= max(k_y, k_z)           */
    int k_y, k_z;       /* multistep orders K_y, K_z in [1, 6] (Tables 1-2)       */
    int L;              /* Gauss-Hermite points, 1..64 (eq (21))                 */
    int n_x[2];         /* grid points per axis, >= 4 (x_i = x_min + i dx)       */
    double x_min[2], x_max[2];
    double drift[2];    /* X_{t+h} = X_t + drift h + vol (W_{t+h} - W_t)          */
    double vol[2][2];   /* row-major; d = 1 uses vol[0][0]; d = 2 needs
                           vol[0][0], vol[1][1] > 0 (and vol[0][1] = 0, i.e. a
                           lower-triangular factor, for the 2-D kernels)         */
    double drift_x;     /* d = 1: forward coefficients of eq (1) that depend on
                           the state, a(x) = drift[0] + drift_x x and
                           b(x) = vol[0][0] + vol_x x, b > 0 over the grid; the
                           node of layer n+j is one Euler step over j dt,
                           x + a(x) j dt + b(x) sqrt(2 j dt) a_l, located per
                           grid point.  Both 0 (the usual case): constant
                           coefficients, drift[0] and vol[0][0] > 0.  d = 2: 0 */
    double vol_x;
    int driver;         /* bsde_driver_kind                                      */
    double p[8];        /* driver parameters                                     */
    int picard_max;     /* Picard iterations, >= 1                               */
    double picard_tol;  /* > 0: stop a point when |dy| <= tol max(1, |y|);
                           <= 0: exactly picard_max iterations                   */
    int prec;           /* bsde_precision                                        */
    int n_stop;         /* last layer computed, 0 <= n_stop <= N - K; 0 is the
                           full sweep.  A larger value stops early (a checkpoint
                           of the backward loop) and y0, z0 then receive layer
                           n_stop.                                               */
    int z_form;         /* bsde_z_form                                           */
    int quad;           /* bsde_quad                                             */
    int interp;         /* bsde_interp                                           */
    const double *coef_tab; /* d = 1, optional: forward coefficients of eq (1)
                           of any form, tabulated on the grid (host memory,
                           copied by bsde_plan, read nowhere else):
                           2 * tab_steps * n_x[0] doubles, row s holding
                           a(t, x_i) at [2 s n_x + i] and b(t, x_i) > 0 at
                           [(2 s + 1) n_x + i].  The node of layer n+j from
                           x_i is the Euler step x_i + a j dt + b sqrt(2 j dt)
                           a_l with the row s = n (tab_steps = n_t: a and b
                           at t_n) or s = 0 (tab_steps = 1: time-homogeneous).
                           drift[0], vol[0][0], drift_x and vol_x are then
                           not used (the slopes must be 0).  NULL with
                           tab_steps = 0: the coefficients above.            */
    int tab_steps;      /* 0, 1 or n_t                                           */
} bsde_problem;

/* Largest stability ratio R = vol sqrt(2 dt) / dx (Gauss-Hermite spread of
 * one step, in grid cells) at which the scheme of eq (20) with the
 * Gauss-Hermite expectations of eq (21) and the natural spline was found
 * linearly stable for K <= 6 and L in {16, 32} (a von Neumann analysis of
 * the scheme for linear drivers on the uniform grid).  At larger R the
 * quadrature aliases grid-scale modes and rounding noise can grow without
 * bound over the steps; such problems still run (bsde_problem_info flags
 * them). */
#define BSDE_STABILITY_LIMIT 16.0

typedef struct {
    double stability_ratio; /* R; d = 2: the larger of the two axes'          */
    int stable;             /* 1 when R <= BSDE_STABILITY_LIMIT (to a relative
                               1e-12, the rounding of R itself)               */
    int K;                  /* max(k_y, k_z): layers kept and initial layers  */
    int node_reach;         /* widest node offset from a grid point, in cells */
    int supported;          /* 1 when bsde_plan implements the problem        */
} bsde_problem_info_t;

/*
 * bsde_problem_info -- host-only check of one problem (no device call): the
 * validation bsde_plan applies, and the plan-time quantities that decide how
 * well the scheme behaves on it, chiefly the stability ratio and its flag.
 * Errors: BSDE_EINVAL for an invalid problem or NULL pointer.
 */
bsde_status bsde_problem_info(const bsde_problem *pb, bsde_problem_info_t *info);

/* Opaque, immutable after creation.  A plan may be shared by threads, but
 * solves that use one workspace must not overlap. */
typedef struct bsde_plan_s *bsde_plan_t;

typedef struct {
    int picard_iter_max;           /* largest Picard count over all points/steps */
    double picard_iter_mean;       /* mean Picard count per point-step            */
    long long picard_nonconverged; /* point-steps that hit picard_max (tol mode)  */
    long long nonfinite;           /* non-finite y or z values in the output      */
    double stability_ratio;        /* largest R = vol sqrt(2 dt) / dx over the
                                      instances (Gauss-Hermite spread per cell)   */
    int unstable_instances;        /* instances with R > BSDE_STABILITY_LIMIT     */
    float elapsed_ms;              /* device time of the solve (hipEvents)        */
} bsde_stats;

/* Per-instance buffers of a batched solve (all device pointers). */
typedef struct {
    const double *init_y; /* K x n_x: layer r at t_{N-K+1+r}, r = 0..K-1         */
    const double *init_z; /* K x n_x                                             */
    double *y0;           /* n_x: y at t_0 on the grid                           */
    double *z0;           /* n_x: z at t_0 on the grid                           */
} bsde_io;

/*
 * bsde_plan -- validate `batch` problems at pb[0..batch-1] and build their
 * plan: Gauss-Hermite nodes and weights (eq (21), Golub-Welsch), the
 * coefficients of Tables 1 and 2 (not-a-knot spline integrals, Section 2.1),
 * and for every j = 1..K and node l the shifted-node offset on the uniform
 * grid split into an integer cell and a fraction (Section 3.2, O(1)
 * location), with the spline basis weights at that fraction.  Small constant
 * tables are copied to the current device.
 * Errors: BSDE_EINVAL for an invalid problem, batch < 1, or problems of
 * different d in one batch; BSDE_EUNSUPPORTED for a d = 2 problem with
 * vol[0][1] != 0, a driver other than BSDE_DRIVER_LINEAR, the FP32 form
 * with BSDE_ZFORM_YDW, exact expectations or state-dependent coefficients,
 * or nodes of one axis-0 row spread over more than 240 cells along axis 1
 * (the sweep's LDS window), and for a d = 1 grid whose ring plane would reach 4 GiB (about 2.7e8 points
 * in FP64, 5.4e8 in FP32); BSDE_ENOMEM, BSDE_EDEVICE.  *out is set only on
 * success.
 */
bsde_status bsde_plan(const bsde_problem *pb, int batch, bsde_plan_t *out);

/* Release a plan and its device tables (NULL is a no-op). */
void bsde_plan_destroy(bsde_plan_t plan);

/*
 * bsde_workspace_bytes -- size of the caller-owned device workspace a solve
 * with this plan needs: the ring of K + 1 time layers (y, its spline second
 * derivatives, z, its second derivatives, ghost-padded), accumulators and
 * statistics.  0 on a NULL plan.
 */
size_t bsde_workspace_bytes(bsde_plan_t plan);

/*
 * bsde_solve -- run the backward sweep of eq (20) for instance 0 of the plan:
 * for n = N-K, ..., 0 and every grid point, the Gauss-Hermite expectations of
 * the spline-interpolated layers n+1..n+K, the explicit z^n, the Picard solve
 * of the implicit y^n, and the natural spline of the new layer.
 *   ws      device workspace of at least bsde_workspace_bytes(plan) bytes,
 *           256-byte aligned; its contents on entry do not matter.
 *   init_y  device, K x n_x doubles: row r is y at t_{N-K+1+r} (row K-1 is the
 *           terminal layer g(x_i)); K = max(k_y, k_z).  For d = 2 a row is
 *           the n_x[0] x n_x[1] grid, point (i0, i1) at i0 n_x[1] + i1.
 *   init_z  device, K x n_x doubles, same layout for z; for d = 2 each row r
 *           is two grid rows, z_1 then z_2.
 *   y0, z0  device, n_x doubles each: receive y and z at t_0 on the grid
 *           (d = 2: y0 one grid, z0 two grids, z_1 then z_2).
 *   stream  hipStream_t or NULL.
 *   st      NULL: fully asynchronous.  Non-NULL: the call synchronises the
 *           stream, fills *st and returns BSDE_ENOCONV / BSDE_ENONFINITE when
 *           those counts are non-zero (outputs are written in both cases).
 * The kernels of one solve are captured once per (workspace, buffers,
 * statistics flag) into a hipGraph held by the plan (at most 4 are kept);
 * later solves with the same buffers replay it as a single launch.  Set the
 * environment variable BSDE_GRAPH=0 before bsde_plan to launch directly.
 * Errors: BSDE_EINVAL (NULL pointer, misaligned workspace), BSDE_EDEVICE.
 */
bsde_status bsde_solve(bsde_plan_t plan, void *ws, const double *init_y, const double *init_z,
                       double *y0, double *z0, void *stream, bsde_stats *st);

/*
 * bsde_solve_batched -- bsde_solve for every instance b of a plan (any batch
 * size; instances may differ in every field except d), with io[b] (host
 * array of `batch` entries holding device pointers) giving the buffers of
 * instance b, laid out as in bsde_solve.  One workspace serves the whole
 * batch.  Instances of equal precision and driver form a group; each time
 * step is one kernel launch per group that advances every instance of the
 * group still active by one layer (instances of fewer steps finish first).
 * The whole solve is one hipGraph launch as for bsde_solve.  Stats, when
 * requested, aggregate over the batch.
 * The graph is a chain of per-step launches, not one persistent kernel: the
 * kernel boundary is the step's device-wide barrier, while a persistent
 * kernel whose tiles waited on their neighbours through device-scope flags
 * ran 2.5 times slower (each release/acquire pair writes back and
 * invalidates the L2 caches).  It is captured on the first solve with a
 * given set of buffers (the plan does not know them) and replayed by later
 * solves with the same buffers.
 * Errors: as bsde_solve.
 */
bsde_status bsde_solve_batched(bsde_plan_t plan, void *ws, const bsde_io *io, void *stream,
                               bsde_stats *st);

/*
 * bsde_initial_layers -- Section 3.1 step 2: the K - 1 initial layers that
 * follow the terminal one (K = max(k_y, k_z)), computed on the device by the
 * 1-step scheme (eq (20) with K_y = K_z = 1, row 1 of Tables 1 and 2) with
 * `substeps` steps per dt = T / n_t: layer t_{N-r} is the 1-step sweep from
 * t_{N-r+1} over substeps steps of dt / substeps, r = 1..K-1, through the
 * same sweep kernels as bsde_solve (the driver sees the absolute times).
 * The 1-step scheme's z is first order in its step (Theorem 2), so the
 * initial layers' error falls like 1/substeps.
 *   pb        the problem of the main solve (its n_stop is ignored).
 *   substeps  >= 1.
 *   ws        device workspace of ws_bytes bytes, 256-byte aligned; the
 *             workspace of a plan of pb (bsde_workspace_bytes) is large
 *             enough whenever K >= 2.
 *   init_y, init_z  device, laid out as for bsde_solve; on entry row K-1
 *             holds the terminal layer; on return rows 0..K-2 hold the layers
 *             at t_{N-K+1}..t_{N-1} (row K-1 is unchanged).
 *   stream    hipStream_t or NULL; the call synchronises it.
 * Plans one K = 1 problem per layer (host tables and small device tables).
 * Errors: BSDE_EINVAL (invalid problem, NULL pointer, substeps < 1, a
 * workspace too small), the errors of bsde_plan and bsde_solve.
 */
bsde_status bsde_initial_layers(const bsde_problem *pb, int substeps, void *ws, size_t ws_bytes,
                                double *init_y, double *init_z, void *stream);

/*
 * bsde_checkpoint_layers -- resume data of a solve stopped at a checkpoint
 * (Section 3.1 step 3's backward loop cut at layer n_stop): after
 * bsde_solve / bsde_solve_batched of `plan` with workspace `ws` has finished
 * (and before ws is used again), writes layers n_stop .. n_stop + K - 1 of
 * instance b (K = max(k_y, k_z)) to layers_y and layers_z in the layout of
 * init_y / init_z: row r = layer n_stop + r (d = 1: K x n_x and K x n_x;
 * d = 2: K x n_x[0] n_x[1] and K x 2 x n_x[0] n_x[1]), caller-owned device
 * buffers.  A problem with n_t' = n_stop + K - 1 and T' = n_t' T / n_t (same
 * dt, same absolute times; a per-step coefficient table keeps its first n_t'
 * rows) started from them continues the sweep: it gives
 * the layers of the uninterrupted solve (the FP32 form exports each stored
 * value plus its rounding residual, which the resumed solve splits back into
 * the same pair).  Asynchronous on the stream.
 * Errors: BSDE_EINVAL (NULL pointer, b outside the batch), BSDE_EDEVICE.
 */
bsde_status bsde_checkpoint_layers(bsde_plan_t plan, void *ws, int b, double *layers_y,
                                   double *layers_z, void *stream);

/* Size of the library's static device workspace (64 MiB per GPU). */
#define BSDE_STATIC_WORKSPACE_BYTES (((size_t)64) << 20)

/*
 * bsde_solve_batched_static -- for callers that cannot allocate device memory
 * (code under hipGraph stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): bsde_solve_batched without the statistics, with the
 * plan's workspace taken from a static device array of the library
 * (BSDE_STATIC_WORKSPACE_BYTES, one per GPU, held until the process ends)
 * instead of a caller-owned buffer.  Allocates nothing: no hipMalloc,
 * hipFree, event, graph or host allocation; it only enqueues the solve's
 * kernels on the stream (asynchronously).  The caller still owns the inputs
 * and outputs (io as for bsde_solve_batched).
 * Every call on one GPU uses that GPU's one static workspace: calls whose
 * work overlaps on a GPU (different streams or threads without ordering)
 * race and give wrong results.  A solve initialises everything it reads, so
 * a call does not depend on the previous call's contents.
 * The plan must have been made on the current device.
 * Errors: BSDE_EINVAL (NULL pointer, another current device),
 * BSDE_ESCRATCH (bsde_workspace_bytes(plan) > BSDE_STATIC_WORKSPACE_BYTES),
 * BSDE_EDEVICE.
 */
bsde_status bsde_solve_batched_static(bsde_plan_t plan, const bsde_io *io, void *stream);

/* Per-kernel device time of one solve, from hipEvent pairs around launches. */
typedef struct {
    double sweep_ms;      /* summed duration of the sweep launches (one per step
                             and group, with the launch that adds a split
                             sweep's partial sums)                              */
    int sweep_launches;
    double spline_ms;     /* summed duration of the separate spline launches of
                             the loop (0 launches when the sweep's own kernels
                             build the splines: fused windows, split Toeplitz) */
    int spline_launches;
    int path;             /* sweep kernel of group 0: 0 = LDS-staged windows with
                             the spline of the newest layer in-kernel, 1 = direct
                             loads, 2 = the two-dimensional sweep, 3 = nodes
                             located per point (state-dependent coefficients),
                             4 = exact expectations as banded Toeplitz products
                             on matrix cores (BSDE_QUAD_EXACT)                   */
    int points_per_lane;  /* grid points per lane of the sweep kernel            */
    int node_groups;      /* thread groups sharing the nodes of one tile; for
                             paths 1 and 4 the blocks that split one tile's node
                             chunks or band (their partial sums are added by a
                             second launch when > 1)                             */
    int blocks;           /* tiles of the first sweep launch of group 0          */
    long long lds_bytes;  /* dynamic LDS per block of the sweep kernel           */
} bsde_kernel_times;

/*
 * bsde_profile_kernels -- bsde_solve_batched (same arguments, same results)
 * launched directly, with a hipEvent pair recorded around every launch of the
 * sweep and spline kernels of the backward loop, so their average durations
 * can be set against their algorithmic work.  Synchronises the stream and
 * fills *kt.  Meant for measurement; bsde_solve is the fast path.
 * Errors: as bsde_solve.
 */
bsde_status bsde_profile_kernels(bsde_plan_t plan, void *ws, const bsde_io *io, void *stream,
                                 bsde_kernel_times *kt);

typedef struct {
    int path, points_per_lane, node_groups;  /* chosen shape of group 0           */
    double best_ms_per_step;                 /* its measured time of one step      */
    int candidates;                          /* shapes timed over all groups       */
} bsde_tune_report;

/*
 * bsde_autotune -- choose the sweep kernel shape of every group of the plan
 * by measurement: the initial layers of io are loaded into ws, and for each
 * shape that fits (fused kernel with 1, 2 or 4 points per lane and 1 or 2
 * node groups; when none fits, the direct kernel with one point per lane,
 * split over blocks on a small grid, and with two) the group's first time step
 * and three more spread over its steps (so a batch's shrinking set of active
 * instances counts) are run `reps` times, replayed from a captured graph as
 * a solve would run them (directly when BSDE_GRAPH=0), and timed with
 * hipEvents, in two passes over the shapes (each keeps its faster pass); the
 * fastest shape is kept in the plan.  Replaces the default shape (or BSDE_SWEEP); drops the
 * plan's captured graphs.  Synchronises the stream.  Must not run while
 * another solve uses the plan.  rep may be NULL.
 * Errors: BSDE_EINVAL (as bsde_solve_batched, or reps < 1), BSDE_EDEVICE.
 */
bsde_status bsde_autotune(bsde_plan_t plan, void *ws, const bsde_io *io, void *stream, int reps,
                          bsde_tune_report *rep);

/* Gauss-Hermite rule (nodes ascending, weights for exp(-x^2), sum sqrt(pi))
 * as used by the plan; L in [1, 64].  Host arrays of L doubles. */
bsde_status bsde_gauss_hermite(int L, double *a, double *w);

/* Row K (1..6) of Table 1 (table = 1: gamma^K_{K,j}, integral over K steps
 * divided by K dt) or Table 2 (table = 2: integral over the first step divided
 * by dt) into g[0..K]: the not-a-knot spline quadrature weights. */
bsde_status bsde_gamma(int table, int K, double *g);

/* Human-readable name of a status code (static storage). */
const char *bsde_status_string(bsde_status s);

#ifdef __cplusplus
}
#endif
#endif /* BSDE_H */
