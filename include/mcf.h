/*
 * mcf.h -- C ABI of libmcf, an MI355X (gfx950) PDHG solver for the
 * destination-aggregated all-pairs multicommodity network flow problem
 * (Zhang & Boyd, "Solving Large Multicommodity Network Flow Problems on GPUs",
 * arXiv 2501.17996).
 *
 * Problem (Section 1.1, (e-prob)/(e-compact-prob)): maximize U(T) = sum_{i!=j} u_ij(T_ij)
 * over the destination-based flow F (n x m, F_il = flow on edge l destined to node i)
 * subject to F >= 0, F^T 1 <= c and T = -F A^T, where A is the incidence matrix
 * (A[head(l), l] = +1, A[tail(l), l] = -1) and T_ij is the traffic from j to i.
 * Method: Algorithm 2.1 (PDMCF): the over-relaxed PDHG step (e-pdhg-step), the
 * projection onto {f >= 0, 1^T f <= c_l} per edge column (Section 2.3), the dual
 * proximal operators of the log and power utilities (Section 2.3), the adaptive
 * primal weight (e-primal_weight) and eta = 1/sqrt(2 d_max) (e-eta).
 *
 * Conventions for every function:
 *   - every call returns int: MCF_OK (0) or a negative MCF_E_* code; nothing
 *     throws or aborts; mcf_strerror() names a code;
 *   - host arrays are plain host pointers; the library copies what it needs, so
 *     callers may free inputs on return;
 *   - device memory belongs to the handle, or lives inside the caller's workspace
 *     (mcf_options.workspace, e.g. a torch tensor's data pointer) when one is given;
 *   - a handle is used by one host thread at a time; handles are independent.
 *
 * Layouts (host side, always FP64 even when the iterates are FP32):
 *   F: n*m, F[l*n + i] = flow on user edge l destined to node i;
 *   T, Y, w: n*n, X[j*n + i] = entry (i, j); w[j*n+i] weights the traffic j -> i.
 */
#ifndef MCF_H
#define MCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcf_solver mcf_solver; /* opaque; owns its device buffers */

/* Utilities (Section 1.1 allows any strictly concave increasing u on s > 0; Section 2.3 solves
 * the one-dimensional dual prox for it in general):
 *   LOG    u = w log s;
 *   POWER  u = w s^gamma, gamma in (0, 1);
 *   ALPHA  the alpha-fair family u = w s^(1-alpha) / (1-alpha), 0 < alpha <= 16, alpha != 1
 *          (alpha > 1 gives negative utilities that penalise small traffic more; LOG is its
 *          limit alpha -> 1, and alpha = 1 - gamma with weight w gamma is POWER). */
enum { MCF_UTIL_LOG = 0, MCF_UTIL_POWER = 1, MCF_UTIL_ALPHA = 2 };
enum { MCF_FP64 = 0, MCF_FP32 = 1 };                     /* precision of F, Y; reductions are always FP64 */
enum { MCF_STOP_REL_KKT = 0, MCF_STOP_PAPER = 1 };       /* rel_kkt <= tol  |  r^k < n m tol (Algorithm 2.1) */
enum { MCF_OK = 0, MCF_E_ARG = -1, MCF_E_GRAPH = -2, MCF_E_NOMEM = -3, MCF_E_DEVICE = -4, MCF_E_STATE = -5 };
enum { MCF_RUNNING = 0, MCF_CONVERGED = 1, MCF_MAX_ITER = 2, MCF_DIVERGED = 3 }; /* solve states, not errors */
/* Kernel organisation of one iteration.  TWO_PHASE: an edge-phase launch then a node-phase
 * launch.  FUSED (n <= 512 only): one launch in which each node's workgroup projects every
 * edge incident to it.  Both compute the same iteration; AUTO picks FUSED when n <= 512. */
enum { MCF_KERNELS_AUTO = 0, MCF_KERNELS_TWO_PHASE = 1, MCF_KERNELS_FUSED = 2 };

/* Solver options.  Defaults (mcf_options_default) are the paper's parameters:
 * rho = 1.9 (Section 2.2), theta = 0.5, k_adapt = 100, tau = 1e-5, omega0 = 1 (Section 2.4). */
typedef struct {
    double tol;             /* stopping tolerance, > 0 (meaning set by stop_rule) */
    int64_t max_iter;       /* iteration limit (total, counted from the cold start) */
    int32_t precision;      /* MCF_FP64 or MCF_FP32 */
    int32_t stop_rule;      /* MCF_STOP_REL_KKT or MCF_STOP_PAPER */
    int32_t check_every;    /* residual evaluated every check_every iterations (>= 1) and at the last one */
    int32_t k_adapt;        /* adapt omega when k is a multiple of k_adapt (k = 0 included); <= 0 disables */
    double rho, theta, tau, omega0;
    int32_t device;         /* HIP device ordinal */
    int32_t kernel_mode;    /* MCF_KERNELS_AUTO (fused for n <= 512), MCF_KERNELS_TWO_PHASE or MCF_KERNELS_FUSED */
    void *stream;           /* hipStream_t to run on, or NULL for a stream owned by the handle */
    void *workspace;        /* optional caller device memory (>= mcf_workspace_bytes), or NULL */
    size_t workspace_bytes;
    int64_t adapt_until;    /* omega is adapted only while k < adapt_until (-1: always).  Section 2.4 notes that
                               freezing omega after some iterations restores the constant-omega convergence proof */
    /* Launch shape of the two-phase iteration; 0 = the measured choice for this n and precision
     * (the table tune.py writes).  edge_waves: 1 = one wave per out-edge, eight out-edges of a
     * tail at once; -1 = one wave per edge over a flat grid of eight-edge workgroups, the
     * out-edge sums of F A^T gathered by the node phase; 4, 8 or 16 = that many waves per edge
     * column, the out-edges of a tail in turn.
     * edge_vectors: 16-byte vectors per lane of a column.  The pair must be one that
     * mcf_edge_shapes lists and whose columns hold n entries (64 * waves * vectors * 16 / size
     * of the iterate), else MCF_E_ARG; both or neither are given.  node_block: 64 or 256
     * threads per node-phase block.  Results depend on the shape only through the order of
     * floating-point sums. */
    int32_t edge_waves, edge_vectors, node_block;
    /* 1 (default): each block of check_every iterations is captured once per block shape into a
     * HIP graph and replayed, which shortens the gap between dependent launches; 0: launched one
     * by one.  Results are the same either way.  With kernel timing on (mcf_enable_kernel_timing),
     * blocks are still replayed from their graphs and one pair of events spans each solve or run. */
    int32_t graphs;
    /* Form of the regular two-phase node launch: 0 (default) = chosen from the size of F (the
     * latency form while F is at most 512 MiB, else the streaming form); 1 = latency form (the
     * entry's own operands and a whole batch of in-edge loads in flight at once); 2 = streaming
     * form (fewer loads in flight per wave).  Other values: MCF_E_ARG.  The two forms compute the
     * same operations in the same order, so results are bitwise the same. */
    int32_t node_form;
} mcf_options;

/* Latest solve record.  Residuals are those of the last checked iteration:
 *   r          the residual r(Q^k) of (e-res) (+inf while T^ is not positive off the diagonal);
 *   r_paper    r / (n m), compared with tol by MCF_STOP_PAPER;
 *   rel_primal ||offdiag(T(Y^k) - T^)||_F / ||offdiag T^||_F, T(Y) the traffic the prices Y ask for;
 *   rel_dual   sqrt(r / ||G||_F^2) with G = U'A;
 *   rel_gap    (p - d) / (1 + |p| + |d|), p = -U(T^), d the dual objective of the reduced Lagrangian (e-L);
 *   rel_kkt    max(rel_primal, rel_dual, rel_gap), +inf unless T^ > 0 and Y^k < 0 off the diagonal. */
typedef struct {
    int32_t state;          /* MCF_RUNNING / CONVERGED / MAX_ITER / DIVERGED */
    int32_t checked;        /* 1 if the residual fields belong to the last iteration */
    int64_t iters;          /* PDHG iterations performed since the cold start */
    double r, r_paper, rel_primal, rel_dual, rel_gap, rel_kkt;
    double primal_obj, dual_obj, infeasible_frac;
    double omega, alpha, beta, delta_f, delta_y;
    double seconds;         /* wall time of the last mcf_solve / mcf_run call */
} mcf_result;

/* Resumable scalar state (Section 2.5 warm start): iteration k and primal weight omega.  alpha and
 * beta (the step sizes eta/omega and eta*omega, Section 2.4) and r (the residual of the last
 * checked iteration) are reported by mcf_get_state; mcf_set_state reads only k and omega. */
typedef struct {
    int64_t k;
    double omega;
    double alpha, beta, r;
} mcf_scalars;

/* Fills *o with the defaults: tol 1e-4, REL_KKT, FP64, check_every 1, max_iter 100000,
 * k_adapt 100, rho 1.9, theta 0.5, tau 1e-5, omega0 1, adapt_until -1, device 0, no stream,
 * no workspace, measured launch shapes, graphs 1. */
void mcf_options_default(mcf_options *o);

/* Device bytes one instance needs at this precision with the kernel organisation AUTO picks
 * (buffers, CSR lists, partials).  Returns 0 if n or m is out of range. */
size_t mcf_workspace_bytes(int32_t n, int32_t m, int32_t precision);

/* Builds an instance and sets the cold start of Section 2.5 (F = 0, Y = I - 1 1^T, omega = omega0).
 *   n, m       nodes (2 <= n <= 16384) and edges (m >= 1);
 *   tail, head m edge endpoints in [0, n), tail != head (parallel edges allowed);
 *   cap        m capacities c_l > 0 (Section 1.1);
 *   utility    MCF_UTIL_LOG, MCF_UTIL_POWER or MCF_UTIL_ALPHA; gamma is the power utility's gamma
 *              (0 < gamma < 1) or the alpha-fair alpha (0 < alpha <= 16, alpha != 1); ignored for LOG;
 *   w          n*n weights, w[j*n+i] > 0 for i != j (diagonal ignored);
 *   opt        options or NULL for the defaults.
 * Errors: MCF_E_ARG for any range/positivity/NULL violation or tol <= 0; MCF_E_GRAPH if the
 * graph is not strongly connected (Section 1.1 requires a path between every pair);
 * MCF_E_NOMEM / MCF_E_DEVICE for allocation or HIP failures.  *out is NULL on error. */
int mcf_create(int32_t n, int32_t m, const int32_t *tail, const int32_t *head, const double *cap,
               int32_t utility, double gamma, const double *w, const mcf_options *opt, mcf_solver **out);

/* Runs Algorithm 2.1 from the current state until the stop rule holds, the iteration
 * count reaches max_iter, or the step norms become non-finite.  Blocking.  Returns MCF_OK
 * whatever the outcome: read the outcome with mcf_status. */
int mcf_solve(mcf_solver *s);

/* mcf_solve without blocking: a host thread of the library runs the same solve on the handle's
 * stream and returns.  Poll mcf_status: its state is MCF_RUNNING, with the record of the latest
 * finished block of check_every iterations, until the solve ends.  Meanwhile every other call on
 * the handle returns MCF_E_STATE (mcf_status and mcf_layout excepted; mcf_destroy stops the solve
 * after its current block and waits for it).  MCF_E_STATE if a solve is already running. */
int mcf_solve_async(mcf_solver *s);

/* Runs exactly `iters` more PDHG iterations with no stop test (residual every check_every
 * iterations and at the last one).  For trajectory comparison and timing. */
int mcf_run(mcf_solver *s, int64_t iters);

/* Restores the cold start (F = 0, Y = I - 1 1^T, omega = omega0, k = 0) on the device. */
int mcf_reset(mcf_solver *s);

/* Copies the latest record into *out.  After an mcf_solve_async that failed, returns its error. */
int mcf_status(const mcf_solver *s, mcf_result *out);

/* Downloads the projected flow Fhat of the last checked iteration (the iterate Algorithm 2.1
 * returns), its traffic T = -Fhat A^T, and the current dual Y.  NULL outputs are skipped. */
int mcf_get_solution(mcf_solver *s, double *F, double *T, double *Y);

/* Downloads the resumable state: F^{k-1/2}, Y^k and the scalars.  NULL outputs are skipped. */
int mcf_get_state(mcf_solver *s, double *F, double *Y, mcf_scalars *sc);

/* Uploads a state (warm start or resume).  F may not be NULL; Y and sc may be NULL to keep
 * the current ones.  Values are rounded to the iterate precision. */
int mcf_set_state(mcf_solver *s, const double *F, const double *Y, const mcf_scalars *sc);

/* Releases the handle and its device memory.  NULL-safe. */
void mcf_destroy(mcf_solver *s);

/* Static text for a return code. */
const char *mcf_strerror(int code);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): mcf_create + mcf_solve + mcf_get_solution + mcf_status + mcf_destroy in one blocking
 * call that allocates nothing.  Its workspace is a static device array of MCF_STATIC_BYTES per
 * GPU, which the library holds until the process ends; the call makes no device or pinned
 * allocation and creates no stream, event or graph (host memory is used for the CSR build).
 *   arguments  as mcf_create, and the outputs of mcf_get_solution (F, T, Y: host FP64, NULL
 *              skipped) and mcf_status (*result, required);
 *   opt        NULL for the defaults; opt->stream is the stream to run on (NULL: the null
 *              stream); opt->workspace must be NULL and workspace_bytes 0; graphs are not used.
 * Errors: those of mcf_create, and MCF_E_ARG when the instance needs more than MCF_STATIC_BYTES
 * (mcf_workspace_bytes gives the need; config2 takes about 10 MB in FP32, 20 MB in FP64).
 * Every call on one GPU shares that GPU's array: calls from threads of one process are
 * serialised by the library, but calls that overlap on one GPU from other processes, or that
 * run on other streams while a call is in flight, race.  Results equal those of the handle
 * API on the same instance and options. */
enum { MCF_STATIC_BYTES = 64 << 20 };
int mcf_solve_static(int32_t n, int32_t m, const int32_t *tail, const int32_t *head, const double *cap,
                     int32_t utility, double gamma, const double *w, const mcf_options *opt, double *F, double *T,
                     double *Y, mcf_result *result);

/* Test hook: writes a NaN into F (which = 0, flat user index l*n+i) or Y (which = 1,
 * j*n+i) on the device; the next iteration then reports MCF_DIVERGED. */
int mcf_debug_poison(mcf_solver *s, int32_t which, int64_t index);

/* Kernel timing for the roofline of the iteration, on the solver's stream, while enabled.
 * With graphs (the default) one pair of HIP events spans each mcf_solve / mcf_run: every launch
 * of its iterations, checks and control included.  Without, events recorded by the dispatches bracket
 * the single launch of a fused iteration, or the edge and node launches of a two-phase one, in
 * every 7th iteration (7 is prime to the usual check and adapt periods, so the sample keeps their
 * mix).  mcf_kernel_time returns the summed milliseconds and the number of iterations they
 * cover since the last enable. */
int mcf_enable_kernel_timing(mcf_solver *s, int32_t enable);
int mcf_kernel_time(mcf_solver *s, double *edge_ms, int64_t *edge_launches);

/* The two-phase edge shapes compiled into the library for this precision: writes up to cap
 * (waves, vectors) pairs (waves 1 = the concurrent form, -1 = the flat form) and returns how
 * many there are (0 for an invalid precision). */
int32_t mcf_edge_shapes(int32_t precision, int32_t *waves, int32_t *vectors, int32_t cap);

/* Internal sizes chosen at create: padded leading dimension, threads per edge column,
 * entries per thread, and the kernel organisation in use (MCF_KERNELS_TWO_PHASE or _FUSED). */
int mcf_layout(const mcf_solver *s, int32_t *ld, int32_t *edge_block, int32_t *edge_ept, int32_t *kernel_mode);

/* ---------------------------------------------------------------- batching pool
 * A pool runs many instances (each created with n <= 512 and the pool's precision) in one
 * stream: every pool iteration performs one PDHG iteration of every active instance, whatever
 * its size or utility: one launch for the instances in the fused iteration, and one edge and
 * one node launch for those in the two-phase iteration, followed on check iterations by one
 * residual and one control launch for all of them.  Each instance follows its own Algorithm 2.1 (its own
 * iteration count, primal weight, adapt schedule and stop test); the residual of every
 * instance is evaluated at the last iteration of each mcf_pool_step.  Instances are admitted
 * and retired between steps (continuous batching); a converged instance stops iterating at
 * once and its slot can be reused after mcf_pool_retire.
 * The pool's iteration counter and work-list sizes live in device memory, and the launch grids
 * are the work counts rounded up (at most 1/8 idle), so a step is replayed from a captured HIP
 * graph whichever instances are admitted; a graph is captured per step length, set of
 * iterations at which some instance adapts omega, and grid.
 * Usage: create solvers (optionally inside caller workspaces), admit them, then repeat
 * { mcf_pool_step; host work; mcf_pool_sync; poll; retire; admit }.  While admitted, a solver
 * answers only mcf_status (the record of the last sync); its other calls return MCF_E_STATE. */
typedef struct mcf_pool mcf_pool;
enum { MCF_POOL_MAX_SLOTS = 256 };

typedef struct {
    int32_t device;         /* HIP device ordinal */
    int32_t precision;      /* MCF_FP32 or MCF_FP64: the precision of every instance admitted */
    size_t hbm_budget;      /* largest sum of mcf_workspace_bytes of the admitted instances (0: no limit) */
    int32_t max_slots;      /* 1 .. MCF_POOL_MAX_SLOTS */
    int32_t check_every;    /* default step length for callers */
    int32_t n_max;          /* largest n admitted, 2 .. 512 (0: 512); it sets the launch shape */
    /* Waves per node workgroup: 8 or (FP32 only) 4, 2 or 1; 0 = the measured choice for n_max and the
     * precision (the table tune.py writes).  Results depend on it only through the order of
     * floating-point sums, and never on which other instances share the pool. */
    int32_t waves;
    int32_t graphs;         /* 1 (default): steps replayed from captured graphs; 0: launched one by one */
    void *stream;           /* hipStream_t or NULL for a stream owned by the pool */
} mcf_pool_options;

/* Fills *o with the defaults: FP32, no budget, 64 slots, check_every 20, n_max 512, measured
 * shape, graphs on, device 0, own stream. */
void mcf_pool_options_default(mcf_pool_options *o);

/* Creates a pool (opt NULL: the defaults).  MCF_E_ARG for an invalid option. */
int mcf_pool_create(const mcf_pool_options *opt, mcf_pool **out);

/* The launch shape in use: waves per node workgroup, the grid of the iteration launch for the
 * instances now admitted, and the largest entries per lane (ceil(n_max / 64) rounded up to 1,
 * 2, 4 or 8). */
int mcf_pool_shape(const mcf_pool *p, int32_t *waves, int32_t *grid, int32_t *max_ept);

/* Sets in *o the precision, kernel organisation and launch shape that an instance of n nodes
 * should be created with to run in this pool: the organisation `tune.py --pool` measured faster
 * in a saturated pool for that size (the fused iteration, or the two-phase one with the flat
 * edge phase and 64-thread node blocks).  Other fields are left as they are.  MCF_E_ARG if n is
 * outside 2 .. n_max. */
int mcf_pool_instance_options(const mcf_pool *p, int32_t n, mcf_options *o);

/* Admits a solver into a free slot.  MCF_E_NOMEM when no slot is free or the budget would be
 * exceeded (retry after a retire); MCF_E_ARG when the solver is already pooled, has another
 * precision, has more than n_max nodes, or uses the two-phase iteration in another form than
 * the flat edge phase with at most 4 vectors per lane and 64-thread node blocks (the form
 * mcf_pool_instance_options gives); MCF_E_STATE when it
 * has converged or diverged.  The solver keeps its state and continues from its current
 * iteration. */
int mcf_pool_admit(mcf_pool *p, mcf_solver *s, int32_t *slot);

/* Enqueues `iters` pool iterations (the last one checks every instance) and returns without
 * waiting.  Waits first for a step still in flight. */
int mcf_pool_step(mcf_pool *p, int32_t iters);

/* Waits for the step in flight and refreshes every slot's record. */
int mcf_pool_sync(mcf_pool *p);

/* The record of the instance in `slot`, as of the last sync. */
int mcf_pool_poll(mcf_pool *p, int32_t slot, mcf_result *out);

/* Releases a slot (after waiting for the step in flight).  The solver becomes a standalone
 * handle again, at the state it reached in the pool. */
int mcf_pool_retire(mcf_pool *p, int32_t slot);

/* Number of occupied slots, workspace bytes admitted, pool iterations run so far. */
int mcf_pool_info(const mcf_pool *p, int32_t *active, size_t *used_bytes, int64_t *iterations);

/* Retires every slot and releases the pool.  NULL-safe. */
void mcf_pool_destroy(mcf_pool *p);

#ifdef __cplusplus
}
#endif

#endif /* MCF_H */
