/*
 * sgweno.h -- C ABI of libsgweno, the MI355X (gfx950) implementation of the
 * sparse-grid fifth-order WENO method of Zhu & Zhang, "Fast sparse grid
 * simulations of fifth order WENO scheme for high dimensional hyperbolic
 * PDEs" (arXiv 2007.10196).
 *
 * The calls follow the paper's algorithm summary (Sec. 2.2.2):
 *   Step 1  restrict the initial condition to the component grids   -> sgw_restrict_initial
 *   Step 2  march every component grid to T with WENO5 + TVD-RK3     -> sgw_advance
 *   Step 3  prolongate every grid to the finest grid and combine    -> sgw_prolongate_combine
 * plus the error norms of Sec. 3 (sgw_exact, sgw_norms), one-launch forms of
 * these steps over many solves (*_many), checkpoints (sgw_snapshot,
 * sgw_restore) and a batched runtime that advances many solves together
 * (sgw_batch_*).
 *
 * Conventions
 *   - Every call returns sgw_status: SGW_OK (0) or a negative error code; the
 *     text of the last error of the calling thread is sgw_last_error().
 *   - The library never allocates device memory.  The caller allocates the
 *     state and scratch buffers with the sizes sgw_plan_footprint reports and
 *     passes device pointers; the library keeps no reference to them after
 *     sgw_solver_free.  Host-side objects (plans, solvers, batches) are owned
 *     by the library and released by the matching *_free call.
 *   - Device work is enqueued on the HIP stream given at creation (NULL means
 *     the null stream) and is asynchronous unless a call says it synchronises.
 *   - A solver must not be used from two host threads at once.
 *   - Arrays on component grids and on the finest grid are row-major with
 *     direction 1 fastest: index = j_1 + n_1 (j_2 + n_2 (j_3 + n_3 j_4)).
 *     Node j of direction k sits at x = lo_k + j h_k, h_k = (hi_k - lo_k)/n_k,
 *     j = 0..n_k-1; beyond either end the values wrap (periodic) or are 0
 *     (sgw_problem.bc).
 *   - Measurement hooks that are not part of the method (stage-launch timing,
 *     VALU issue-rate calibration) are declared in sgweno_measure.h.
 */
#ifndef SGWENO_H
#define SGWENO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGW_MAX_DIM 4

typedef int32_t sgw_status;
#define SGW_OK 0
#define SGW_ERR_INVALID_ARG (-1)   /* an argument is out of range or inconsistent            */
#define SGW_ERR_UNSUPPORTED (-2)   /* valid request the library does not implement           */
#define SGW_ERR_OUT_OF_MEMORY (-3) /* a buffer or budget is too small                        */
#define SGW_ERR_NONFINITE (-4)     /* a wave speed or time step became NaN/Inf on the device */
#define SGW_ERR_HIP (-5)           /* a HIP runtime call failed                              */
#define SGW_ERR_STATE (-6)         /* call out of order (e.g. advance before restrict)       */

/* Flux of eq. (1): u_t + sum_k d/dx_k f_k(u, x) = 0 */
#define SGW_FLUX_ADVECTION 0       /* f_k = a_k u, a_k = flux_params[k]                                 */
#define SGW_FLUX_BURGERS 1         /* f_k = u^2 / 2                                                     */
#define SGW_FLUX_VLASOV_FIXED_E 2  /* dim = 2 m: directions 1..m are x, m+1..2m are v;
                                      f_{x_k} = v_k u, f_{v_k} = E_k(x_k) u with
                                      E_k = flux_params[0] sin(flux_params[1] x_k)                     */
#define SGW_FLUX_VLASOV_HARMONIC 3 /* the same transport with E = -grad |x|^2/2 = -x, the field of the
                                      Vlasov-Boltzmann model (Sec. 3.4, Example 5)                      */
#define SGW_FLUX_VLASOV_MAXWELL 4  /* dim = 3, directions x_2, xi_1, xi_2 (Sec. 3.4, Example 6):
                                      f_{x_2} = xi_2 f, f_{xi_1} = (E_1 + xi_2 B_3) f,
                                      f_{xi_2} = (E_2 - xi_1 B_3) f, with fields E_1, E_2, B_3 of x_2
                                      that every component grid carries at its x_2 nodes and advances
                                      in the same Runge-Kutta stages: B_3' = dE_1/dx_2,
                                      E_1' = dB_3/dx_2 - j_1, E_2' = -j_2 (WENO5 with global LF splitting,
                                      F(B_3, E_1) = (-E_1, -B_3), alpha = 1), currents
                                      j_q = int f xi_q dxi as sums over the grid's velocity nodes times
                                      the velocity cell area; the LF speeds of the xi directions are
                                      the maxima over the grid's nodes of |E_1 + xi_2 B_3| and
                                      |E_2 - xi_1 B_3| of each stage's fields; periodic boundaries */

/* Initial conditions */
#define SGW_IC_SINE 0              /* u0 = p0 + p1 sin(p2 sum_k x_k + p3)                               */
#define SGW_IC_MAXWELL_COS 1       /* f0 = exp(-|v|^2/2) / (2 pi)^(m/2) (1 + p0 prod_k cos(p1 x_k + p_{2+k})) */
#define SGW_IC_VLASOV_BOLTZMANN 2  /* f0 = p0 sin(x_1^2/2)^2 [cos(x_2^2/2)^2] exp(-(|x|^2 + |v|^2)/2), m = 1
                                      [m = 2]; p0 = 1/s normalises the integral (Sec. 3.4, Example 5)   */
#define SGW_IC_VLASOV_MAXWELL 3    /* Example 6, (p0..p5) = (beta, b, delta, v01, v02, k0):
                                      f0 = exp(-xi_2^2/beta) (delta exp(-(xi_1 - v01)^2/beta)
                                           + (1 - delta) exp(-(xi_1 + v02)^2/beta)) / (pi beta),
                                      B_3 = b sin(k0 x_2), E_1 = E_2 = 0                                */

#define SGW_DT_CFL 0               /* dt = cfl / sum_k (A_k / h_k^fine), A_k = max wave speed (Sec. 3) */
#define SGW_DT_POW53 1             /* dt = (min_k h_k^fine)^(5/3), the accuracy-test rule of Sec. 3     */

#define SGW_PROLONG_WENO5 0        /* WENO5 interpolation, eqs. (eqnlnwe), (si), (nlweno)               */
#define SGW_PROLONG_LAGRANGE5 1    /* degree-4 Lagrange interpolation, eq. (lwlag)                      */

#define SGW_FP64 0                 /* state, sweeps and interpolation in FP64                           */
#define SGW_FP32_SWEEP 1           /* state, sweeps and interpolation in FP32; t, dt, the combination
                                      sum and the norms in FP64                                          */

#define SGW_RUN_PLAIN 0            /* one launch per component grid per RK stage, no graph              */
#define SGW_RUN_FUSED 1            /* one launch per RK stage over all component grids; grids that are  */
                                   /* one stage box take all three stages in one launch                 */
#define SGW_RUN_GRAPH 2            /* SGW_RUN_FUSED with each time step captured in a HIP graph         */

/* Boundary condition per direction (the examples of Secs. 3.1-3.3 are periodic;
 * the Vlasov-Boltzmann model of Sec. 3.4, Example 5, prescribes zero boundary
 * values).  Plans with a zero boundary run the stage as line sweeps in every
 * dimension; the prolongation reads 0 beyond the ends as well. */
#define SGW_BC_PERIODIC 0          /* node n_k is node 0                                              */
#define SGW_BC_ZERO 1              /* every value beyond either end (the stencils' ghosts) is 0;
                                      the node at hi_k is one of them                                 */

typedef struct sgw_problem {
    int32_t dim;                   /* 1..4                                                   */
    int32_t flux;                  /* SGW_FLUX_*                                              */
    int32_t ic;                    /* SGW_IC_*                                                */
    int32_t reserved0;             /* must be 0                                               */
    int32_t bc[SGW_MAX_DIM];       /* SGW_BC_* per direction; entries beyond dim are ignored  */
    double lo[SGW_MAX_DIM];        /* domain [lo_k, hi_k)                                     */
    double hi[SGW_MAX_DIM];
    double flux_params[SGW_MAX_DIM];
    double ic_params[8];
    /* Linear relaxation source L(f) = (mu_inf(v) rho(x) - f) / tau of the Vlasov-Boltzmann
       model (Sec. 3.4, Example 5), added to the spatial operator of every Runge-Kutta stage;
       dim = 2 m with directions 1..m = x, m+1..2m = v.  mu_inf(v) = exp(-|v|^2/(2 theta)) /
       (2 pi theta)^(m/2) and rho(x) = int f dv, the sum over the grid's velocity nodes times
       their cell volume, taken from each stage's input.  relax_tau = 0 switches it off; else
       relax_tau > 0 and relax_theta > 0. */
    double relax_tau;
    double relax_theta;
} sgw_problem;

typedef struct sgw_config {
    int32_t root_cells;            /* N_r >= 4: cells per direction of the root grid (Sec. 2.2)   */
    int32_t finest_level;          /* N_L in 0..12                                                 */
    int32_t dt_mode;               /* SGW_DT_*                                                     */
    int32_t prolong;               /* SGW_PROLONG_*                                                */
    int32_t linear_weights;        /* 1: flux weights w_r replaced by d_r (the linear scheme)     */
    int32_t precision;             /* SGW_FP64 or SGW_FP32_SWEEP                                   */
    double cfl;                    /* 0 < cfl <= 1.5 (used in SGW_DT_CFL)                          */
    double eps_flux;               /* epsilon of eq. (2.6); the paper's tables need 1e-3           */
    double eps_interp;             /* epsilon of eq. (eqnlnwe); 1e-3 likewise                      */
    int32_t box[SGW_MAX_DIM];      /* 0: automatic; else the stage-kernel box extent per direction
                                      (must divide every grid's extent in that direction)         */
    int32_t fine_tile[SGW_MAX_DIM];/* 0: automatic; else the prolongation tile per direction       */
    int32_t box_target;            /* 0: automatic (1024); else the largest box (nodes) the
                                      automatic box search may pick, 64..2048                      */
    int32_t blocks_per_cu;         /* 0: as many resident stage workgroups per compute unit as
                                      fit; else at most this many (1..64), a tuning knob         */
    int32_t sweep_form;            /* 3D and 4D stages: 0 automatic (line sweeps, directions 1 and 2
                                      in one launch over whole (x_1, x_2) planes staged in LDS where
                                      every grid's planes fit 2048 nodes, then one launch per
                                      remaining direction); 1 line sweeps, one launch per
                                      direction; 2 stage boxes for 3D (a grid that is one box runs
                                      its three RK stages in one launch: many small 3D solves in a
                                      batch), 4D as 0.  All give the same bits.                   */
} sgw_config;

typedef struct sgw_plan sgw_plan_t;
typedef struct sgw_solver sgw_solver_t;
typedef struct sgw_batch sgw_batch_t;

/* ---------------------------------------------------------------- plans (host only)
 * sgw_plan_create enumerates the component grids of the index set
 * { l : N_L - dim + 1 <= |l| <= N_L } (Sec. 2.2 for 2D, eq. (genformusgc) for
 * general dim), q = N_L - |l| from 0 to dim-1, each q in lexicographic order of
 * (l_1..l_dim), with combination coefficient (-1)^q C(dim-1, q).  Grid l has
 * N_r 2^{l_k} nodes in direction k.  Errors: SGW_ERR_INVALID_ARG for dim
 * outside 1..4, N_r < 4, N_L outside 0..12, cfl outside (0, 1.5], eps <= 0,
 * a Vlasov flux, initial condition or relaxation with odd dim, a negative or
 * non-finite relax_tau, relax_theta <= 0 with relaxation on, a finest grid with more
 * than 2^40 nodes, box_target outside 64..2048, blocks_per_cu outside 0..64,
 * reserved0 not 0 or an unknown boundary condition; SGW_ERR_UNSUPPORTED for a box or
 * tile that does not divide the extents or does not fit one workgroup, and for manual
 * stage boxes with a zero boundary, relaxation or the Vlasov-Maxwell flux (those run as line
 * sweeps), and for the Vlasov-Maxwell flux with a zero boundary.  The Vlasov-Maxwell flux needs
 * dim 3 and its initial condition (SGW_ERR_INVALID_ARG otherwise, also with relaxation).  With
 * fine_tile 0 the prolongation tile is searched over divisors of the finest
 * extent (interpolations, staging, writes and LDS occupancy weighed). */
sgw_status sgw_plan_create(const sgw_problem* problem, const sgw_config* config, sgw_plan_t** out);
void sgw_plan_free(sgw_plan_t* plan);

/* Bytes the caller must provide: state (three copies of every component grid:
 * u^n and the two Runge-Kutta stage buffers), scratch (descriptors, work
 * lists, wave speeds, time-step record, reductions), and the finest-grid FP64
 * output of sgw_prolongate_combine.  Any pointer may be NULL. */
sgw_status sgw_plan_footprint(const sgw_plan_t* plan, uint64_t* state_bytes, uint64_t* scratch_bytes,
                              uint64_t* fine_bytes);

/* Number of grids, component nodes (sum over grids), finest-grid nodes. */
sgw_status sgw_plan_info(const sgw_plan_t* plan, int32_t* num_grids, int64_t* total_nodes,
                         int64_t* fine_nodes);

/* Grid g: level l_k, node counts, coefficient and element offset of its first
 * node inside each state copy (copy u^n starts at byte 0 of the state buffer). */
sgw_status sgw_plan_grid(const sgw_plan_t* plan, int32_t g, int32_t level[SGW_MAX_DIM],
                         int32_t shape[SGW_MAX_DIM], int32_t* coef, int64_t* offset);

/* Vlasov-Maxwell plans: every state copy holds, after the component grids' nodes, the fields of
 * every grid in FP64 (B_3, E_1, E_2 at its x_2 nodes, 3 n_1 values, grids in plan order), from
 * byte offset *offset_bytes of the copy; *count = the number of field values.  Both 0 for other
 * plans.  Copy 0 is u^n (sgw_snapshot and sgw_restore carry the fields with it). */
sgw_status sgw_plan_fields(const sgw_plan_t* plan, uint64_t* offset_bytes, int64_t* count);

/* Finest-grid tile the prolongation kernel uses (one workgroup per tile). */
sgw_status sgw_plan_fine_tile(const sgw_plan_t* plan, int32_t tile[SGW_MAX_DIM]);

/* Number of finest-grid tiles of the prolongation: prod_k N / tile[k]. */
sgw_status sgw_plan_fine_tile_count(const sgw_plan_t* plan, int64_t* count);

/* Box extents the stage kernel uses for grid g (one workgroup per box).  3D and 4D grids
 * without manual boxes (3D: unless sweep_form is 2), and every grid of a plan with a zero
 * boundary, relaxation or the Vlasov-Maxwell flux, march as line sweeps (a lane per segment
 * of a grid line, no boxes) and report all-zero extents. */
sgw_status sgw_plan_grid_box(const sgw_plan_t* plan, int32_t g, int32_t box[SGW_MAX_DIM]);

/* ---------------------------------------------------------------- solvers
 * Binds a plan to caller-owned device memory (at least the footprint sizes,
 * 256-byte aligned) and a HIP stream (hipStream_t passed as void*).  The plan
 * must outlive the solver.  Uploads the grid descriptors (stream-ordered). */
sgw_status sgw_solver_create(sgw_plan_t* plan, void* state_dev, void* scratch_dev, void* hip_stream,
                             sgw_solver_t** out);
void sgw_solver_free(sgw_solver_t* solver);
/* Later calls of this solver enqueue on hip_stream.  Work already enqueued on
 * the previous stream is not waited for: the caller orders it (an event or a
 * synchronisation).  Refused while the solver is in a batch. */
sgw_status sgw_solver_set_stream(sgw_solver_t* solver, void* hip_stream);

/* Alg. Step 1: u^0 = u0 at the nodes of every component grid; t = 0. */
sgw_status sgw_restrict_initial(sgw_solver_t* solver);

/* Alg. Step 2: march every component grid from the current t to t_final with
 * one shared dt per step (Sec. 3: set by the finest spacing, the CFL number
 * and the current wave speed; the last step is clipped to land on t_final).
 * Each step is three TVD-RK3 stages; each stage applies the LF-split WENO5
 * operator of Sec. 2.1 in every direction with the global LF speed of that
 * grid, direction and stage.  mode is SGW_RUN_*.  For state-dependent wave
 * speeds the host polls a device flag every few steps (synchronises). */
sgw_status sgw_advance(sgw_solver_t* solver, double t_final, int32_t mode);

/* Alg. Step 3: out_dev (FP64, (N_r 2^N_L)^dim entries) = sum_g c_g P U_g, with
 * P the dimension-by-dimension WENO5 (or Lagrange5) prolongation of Sec. 2.2.1
 * in increasing direction order; accumulated in FP64 in grid order. */
sgw_status sgw_prolongate_combine(sgw_solver_t* solver, double* out_dev);

/* Step 3 over part of the finest grid: the same values as sgw_prolongate_combine at the
 * finest-grid tiles first_tile .. first_tile + num_tiles - 1 (tiles of the extents
 * sgw_plan_fine_tile reports, numbered with direction 1 fastest; sgw_plan_fine_tile_count
 * gives their number), bitwise; every other entry of out_dev is left as it was.  Calls over
 * ranges that cover every tile once give sgw_prolongate_combine's output, so a caller can
 * spread a large combination over several launches (a serving loop interleaving it with other
 * solves' steps).  SGW_ERR_INVALID_ARG for a range outside 0..count; num_tiles 0 is a no-op. */
sgw_status sgw_prolongate_combine_tiles(sgw_solver_t* solver, double* out_dev, int64_t first_tile,
                                        int64_t num_tiles);

/* Exact solution at time t on the finest grid (FP64), for the error norms:
 * advection: u0(x - a t); Burgers with a sine: characteristics solved by
 * Newton's method (valid before the shock); Vlasov: f0 at the foot of the
 * characteristic, classical RK4 with steps of at most 1e-3.  SGW_ERR_UNSUPPORTED
 * for the Vlasov-Boltzmann model (no closed form). */
sgw_status sgw_exact(sgw_solver_t* solver, double t, double* out_dev);

/* Vlasov-Maxwell (Sec. 3.4, Example 6): out_dev (FP64, 3 N values, N = N_r 2^N_L) = the fields
 * B_3, E_1, E_2 of u^n combined on the finest x_2 grid, sum_g c_g P f_g with P the one-dimensional
 * prolongation of Sec. 2.2.1 along x_2, accumulated in FP64 in grid order.  SGW_ERR_INVALID_ARG for
 * other plans. */
sgw_status sgw_fields_combine(sgw_solver_t* solver, double* out_dev);

/* Entropy functionals of the Vlasov-Boltzmann model (Sec. 3.4, Example 5) of a
 * finest-grid solution f_dev (FP64, the layout sgw_prolongate_combine writes):
 * H_2 = int H^2 M and H_log = int H log(H) M over the domain, H = f / M, with the
 * stationary state M(x, v) = exp(-(|v|^2/2 + |x|^2/2)/theta) / ((2 pi theta)^(m/2)
 * int_x exp(-|x|^2/(2 theta)) dx), the x integral over the x domain in closed form,
 * the others sums over the finest nodes times the cell volume; H log H is 0 where
 * f <= 0.  theta = relax_theta.  Writes result_host[0] = H_2, [1] = H_log in a fixed
 * order (bitwise repeatable); synchronises.  SGW_ERR_INVALID_ARG for odd dim or
 * relax_theta <= 0. */
sgw_status sgw_entropies(sgw_solver_t* solver, const double* f_dev, double* result_host);

/* L1 = mean |a - b|, Linf = max |a - b| over the finest grid, in FP64 and in a
 * fixed order (bitwise repeatable).  Writes result_host[0..1]; synchronises. */
sgw_status sgw_norms(sgw_solver_t* solver, const double* a_dev, const double* b_dev, double* result_host);

/* sgw_norms without the synchronisation: writes L1, Linf to result_dev[0..1]
 * (device memory) in stream order. */
sgw_status sgw_norms_async(sgw_solver_t* solver, const double* a_dev, const double* b_dev, double* result_dev);

/* Alg. Step 3 for many solves in one launch (one workgroup per finest-grid tile
 * of every solve; all solves share dimension and precision; n <= 65535); outs[i]
 * receives solve i's combined solution.  scratch_dev (device, 256-byte aligned)
 * holds the solve list, sgw_prolongate_many_scratch_bytes(solvers, n) bytes.  Runs on
 * hip_stream after the work already enqueued on each solver's own stream that
 * differs from it, and each such stream then waits for the launch (events, no
 * host wait).  Returns without waiting for the device (scratch_dev stays in use
 * until the launch has run in stream order). */
sgw_status sgw_prolongate_combine_many(sgw_solver_t* const* solvers, double* const* outs, int32_t n,
                                       void* scratch_dev, uint64_t scratch_bytes, void* hip_stream);
uint64_t sgw_prolongate_many_scratch_bytes(sgw_solver_t* const* solvers, int32_t n);

/* Alg. Step 1 for many solves in one launch (Sec. 2.2.2): each solve's wave-speed
 * slots and time-step record are cleared, then every grid of every solve gets
 * u0 at its nodes, bitwise as sgw_restrict_initial would.  All solves share a
 * precision.  scratch_dev (device, 256-byte aligned) holds the chunk list,
 * sgw_restrict_many_scratch_bytes(solvers, n) bytes.  Runs on hip_stream after
 * the work already enqueued on each solver's own stream that differs from it,
 * and each such stream then waits for the launch (events, no host wait).
 * Returns without waiting for the device (scratch_dev stays in use until the
 * launch has run). */
sgw_status sgw_restrict_initial_many(sgw_solver_t* const* solvers, int32_t n, void* scratch_dev,
                                     uint64_t scratch_bytes, void* hip_stream);
uint64_t sgw_restrict_many_scratch_bytes(sgw_solver_t* const* solvers, int32_t n);

/* sgw_norms_async for n <= 65535 pairs (a[i], b[i]), each over solve i's finest
 * grid, in one launch: L1 and Linf of pair i go to result_dev[2i], [2i + 1]
 * (device FP64), bitwise as sgw_norms gives them.  scratch_dev (device, 256-byte
 * aligned) holds the pair list and partial sums, sgw_norms_many_scratch_bytes
 * bytes.  Runs on hip_stream after the work already enqueued on each solver's
 * own stream that differs from it (an event); the caller orders other writes of
 * a and b before it.  Returns without waiting for the device (scratch_dev stays
 * in use until the launches have run). */
sgw_status sgw_norms_many(sgw_solver_t* const* solvers, const double* const* a_dev, const double* const* b_dev,
                          int32_t n, double* result_dev, void* scratch_dev, uint64_t scratch_bytes, void* hip_stream);
uint64_t sgw_norms_many_scratch_bytes(sgw_solver_t* const* solvers, int32_t n);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): sgw_norms_many for n <= 32 pairs with
 * no scratch argument and no allocation of any kind.  The pair list and partial
 * sums live in a library-owned device array of sgw_norms_many_static_max_bytes()
 * bytes (about 514 KiB), one per device, held until the process ends.  Results
 * are bitwise those of sgw_norms_many.  Runs on hip_stream only: unlike
 * sgw_norms_many it makes no stream wait on the solvers' own streams, so the
 * caller orders the writes of a and b before it.  Calls on one device share the
 * array: two calls whose launches overlap on one device (different streams, no
 * ordering between them) race and give wrong results.  n above 32 is refused
 * with SGW_ERR_INVALID_ARG.  Returns without waiting for the device. */
sgw_status sgw_norms_many_static(sgw_solver_t* const* solvers, const double* const* a_dev,
                                 const double* const* b_dev, int32_t n, double* result_dev, void* hip_stream);
uint64_t sgw_norms_many_static_max_bytes(void);

/* Current time and number of steps taken; synchronises.  Returns
 * SGW_ERR_NONFINITE if a wave speed or dt became NaN/Inf. */
sgw_status sgw_query(sgw_solver_t* solver, double* t, int64_t* steps);

/* Alg. Step 1 with values the caller samples itself (Sec. 2.2.2): copies the
 * nodes of grid g (solver precision, row-major with direction 1 fastest, the
 * shape sgw_plan_grid reports) from src_dev (device) into u^n, recomputes that
 * grid's wave speed and rewinds the solve to t = 0.  Call it for every grid
 * before sgw_advance; a grid not set keeps its previous values.  Stream-ordered;
 * refused while the solver is in a batch. */
sgw_status sgw_set_grid(sgw_solver_t* solver, int32_t g, const void* src_dev);

/* Checkpoint of a running solve: u^n of every grid, the wave-speed slots and the
 * time record (t, steps, last dt, flags), sgw_snapshot_bytes(solver) bytes of
 * device memory, written or read in stream order.  sgw_restore resumes a solver
 * of the same plan from it (the final time stays the solver's own).  Both are
 * refused (SGW_ERR_STATE) while the solver is in a batch: the batch advances it
 * on the batch stream, so a copy on the solver stream could mix two steps. */
uint64_t sgw_snapshot_bytes(const sgw_solver_t* solver);
sgw_status sgw_snapshot(sgw_solver_t* solver, void* dst_dev);
sgw_status sgw_restore(sgw_solver_t* solver, const void* src_dev);

/* ---------------------------------------------------------------- batches
 * A batch advances the component grids of many solvers together: one fused
 * stage launch per RK stage over the grids of every active solver, each solver
 * with its own t, dt and final time, one HIP graph per step.  All solvers in a
 * batch share the batch's stream and precision.  hbm_budget bounds the sum of
 * the footprints (state + scratch + fine) of the admitted solvers. */
sgw_status sgw_batch_create(int32_t max_solvers, int32_t precision, uint64_t hbm_budget, void* hip_stream,
                            void* scratch_dev, uint64_t scratch_bytes, sgw_batch_t** out);
void sgw_batch_free(sgw_batch_t* batch);
/* Scratch bytes a batch of max_solvers needs for at most max_items stage boxes. */
uint64_t sgw_batch_scratch_bytes(int32_t max_solvers, int64_t max_items);
/* Admit a restricted solver to advance to t_final.  SGW_ERR_OUT_OF_MEMORY when
 * no slot is free or its footprint does not fit the remaining budget;
 * SGW_ERR_UNSUPPORTED for zero-boundary, relaxation and Vlasov-Maxwell solvers, 4D
 * solvers with manual stage boxes, and a 3D solver whose stage form (line sweeps or
 * stage boxes, sweep_form) differs from that of the batch's other 3D solvers (a batch
 * runs its 3D and 4D line sweeps one launch per direction).  Returns without waiting:
 * when the solver's stream differs from the batch stream, the batch stream waits (an
 * event) for the work already enqueued on it. */
sgw_status sgw_batch_admit(sgw_batch_t* batch, sgw_solver_t* solver, double t_final, int32_t* slot);
/* sgw_batch_admit for solvers[0..n) with final times t_final[i]; slots[i]
 * receives each slot.  Stops at the first solver that is refused and returns
 * its error; *n_admitted counts the solvers admitted before it.  The batch
 * stream waits once per distinct solver stream. */
sgw_status sgw_batch_admit_many(sgw_batch_t* batch, sgw_solver_t* const* solvers, int32_t n, const double* t_final,
                                int32_t* slots, int32_t* n_admitted);
/* Advance every active solver by up to nsteps steps (finished ones do nothing).
 * Enqueues graph launches on the batch stream and returns: graphs of 1, 2, 4,
 * ..., 32 steps are captured, and nsteps is launched as its binary
 * decomposition. */
sgw_status sgw_batch_step(sgw_batch_t* batch, int32_t nsteps);
/* Which slots have reached their final time (synchronises).  done_slots has
 * room for max_solvers entries. */
sgw_status sgw_batch_poll(sgw_batch_t* batch, int32_t* done_slots, int32_t* n_done);
/* sgw_batch_poll in two halves, so that steps can be queued while the flags
 * travel: _begin enqueues the gathering of the completion flags at this point of
 * the stream; _end waits for them and reports the slots that were done there.
 * One poll may be in flight (SGW_ERR_STATE otherwise); a slot released or
 * refilled in between is not reported. */
sgw_status sgw_batch_poll_begin(sgw_batch_t* batch);
sgw_status sgw_batch_poll_end(sgw_batch_t* batch, int32_t* done_slots, int32_t* n_done);
/* Remove a solver from the batch; its budget and slot become free.  Returns
 * without waiting for queued steps: a solver whose own stream differs from the
 * batch stream has that stream wait for them (stream-ordered). */
sgw_status sgw_batch_release(sgw_batch_t* batch, int32_t slot);
/* sgw_batch_release for n distinct occupied slots (all checked before any is
 * released).  One event marks the queued steps, and each distinct solver
 * stream waits for it once. */
sgw_status sgw_batch_release_many(sgw_batch_t* batch, const int32_t* slots, int32_t n);
/* Tuning knob: at most blocks_per_cu resident stage workgroups per compute unit
 * (0: as many as fit).  The persistent stage launch splits the box list into
 * equal contiguous ranges over its workgroups, so this trades latency hiding
 * against the share of the last, partly filled round.  Waits for queued steps;
 * the step graph is captured again on the next step. */
sgw_status sgw_batch_set_blocks_per_cu(sgw_batch_t* batch, int32_t blocks_per_cu);
/* Number of stage boxes currently in the batch. */
sgw_status sgw_batch_info(const sgw_batch_t* batch, int32_t* active_solvers, int64_t* boxes, int64_t* nodes);

/* ---------------------------------------------------------------- errors */
const char* sgw_status_string(sgw_status status);
const char* sgw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SGWENO_H */
