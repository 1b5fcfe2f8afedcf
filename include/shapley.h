/*
 * libshapley -- C ABI of an MI355X (gfx950) solver for the Shapley equation
 *
 *     v(x) = max_{a in A(x)} min_{b in B(x,a)} ( sum_y mu p(y|x,a,b) v(y) + r(x,a,b) )
 *
 * of a two-player zero-sum discounted stochastic game with finite state space
 * (Akian & Detournay, "Multigrid methods for two player zero-sum stochastic
 * games", arXiv:1107.1653, Sec. 2, eq. (eq1)), by policy iteration with an
 * algebraic-multigrid inner solve (AMGpi, Sec. 5.1) and by full multilevel
 * policy iteration (FAMGpi, Sec. 5.2, Algorithm algo-FAMGPI).
 *
 * Conventions shared by every entry point
 *   - Return value: SHAPLEY_OK (0) or one of the error codes below; the
 *     message of the last error of the calling thread is returned by
 *     shapley_last_error().  On error no output argument is modified unless
 *     stated otherwise.
 *   - Pointers are host pointers unless a flag says otherwise.  The library
 *     copies every input array; the caller keeps ownership of its arrays.
 *   - A game handle may be used by one thread at a time.  Different handles
 *     may be used concurrently.  shapley_server_submit is thread-safe.
 *   - All computation runs on the HIP device that is current when the handle
 *     is created; work is ordered on the handle's stream.
 */
#ifndef SHAPLEY_H
#define SHAPLEY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define SHAPLEY_OK 0
#define SHAPLEY_EINVAL 1   /* bad sizes, w < 0, row sum > 1 + 1e-12, mu not in (0,1],
                              NaN/Inf, empty action set, bad options */
#define SHAPLEY_ENOMEM 2   /* device allocation failed or budget exceeded */
#define SHAPLEY_ENOCONV 3  /* iteration limits or stagnation; partial results readable */
#define SHAPLEY_EDEVICE 4  /* HIP runtime error or device-side check failure */
#define SHAPLEY_EAGAIN 5   /* result not ready (server) */

/* Message of the last error raised on the calling thread ("" if none). */
const char* shapley_last_error(void);

/* ---------------------------------------------------------------- types */
typedef struct shapley_game_s* shapley_game_t;
typedef struct shapley_server_s* shapley_server_t;

/* Optional geometric description of a game obtained by discretising a PDE on
 * the unit cube (Sec. 3.3): s interior points per side, h = 1/(s+1), states
 * numbered x = (i1-1) + s (i2-1) [+ s^2 (i3-1)].  Needed by FAMGpi for the
 * transfers I (values) and U (strategies) of Sec. 5.2. */
typedef struct shapley_grid {
  int32_t dim;          /* 1, 2 or 3 */
  int32_t s;            /* interior points per side; n must equal s^dim */
  const double* bvals;  /* optional: (s+2)^dim Dirichlet values on the grid
                           extended by its boundary nodes, x1 fastest (only
                           boundary nodes are read); NULL means zero */
} shapley_grid;

enum { SHAPLEY_FP64 = 0, SHAPLEY_MIXED = 1 };
enum { SHAPLEY_AMGPI = 0, SHAPLEY_FAMGPI = 1 };
/* Relaxation of the multigrid cycle (Sec. 4.3: u <- S u + S0 f):
 *   SHAPLEY_SMOOTH_JACOBI  weighted Jacobi, u += omega D^-1 (f - A u)
 *   SHAPLEY_SMOOTH_L1      l1-Jacobi, u += D1^-1 (f - A u) with
 *                          D1_ii = sum_j |a_ij| (no weight)
 *   SHAPLEY_SMOOTH_CF      C/F relaxation (the ordering of the paper's
 *                          smoother, Sec. 6): each sweep relaxes the coarse
 *                          points of the level's C/F splitting, then the fine
 *                          points with the updated coarse values (weighted
 *                          Jacobi within each set) */
enum { SHAPLEY_SMOOTH_JACOBI = 0, SHAPLEY_SMOOTH_L1 = 1, SHAPLEY_SMOOTH_CF = 2 };

/* Solve options.  Fill with shapley_default_opts() first. */
typedef struct shapley_solve_opts {
  double eps;            /* stop when ||F(v) - v||_inf <= eps after a value step
                            (Sec. 5.1); eps = 0 stops when no policy improves
                            (Algorithms algo-MDP / PIalgo). Default 0. */
  int32_t precision;     /* SHAPLEY_FP64: V-cycles in FP64; SHAPLEY_MIXED: FP32
                            V-cycles under FP64 iterative refinement. */
  int32_t method;        /* SHAPLEY_AMGPI, or SHAPLEY_FAMGPI for hierarchies */
  double c_fmg;          /* FAMGpi coarse-level stop eps_l = c_fmg h_l^2 (Sec. 5.2) */
  const int32_t* alpha0; /* optional warm start (host, n entries): MAX policy */
  const int32_t* beta0;  /* optional warm start (host, n entries): MIN policy at alpha0 */
  const double* v0;      /* optional warm start (host, n entries): initial value */
  int32_t max_outer;     /* limit on MAX policy iterations (k) */
  int32_t max_inner;     /* limit on MIN policy iterations per k (n_k) */
  int32_t max_cycles;    /* limit on refinement cycles per linear system */
  double lin_rtol;       /* linear stop ||b - A v||_inf <= lin_rtol max(||b||, ||v||) */
  double lin_atol;       /* ... or <= lin_atol (absolute) */
  double tie_rtol;       /* an incumbent action is kept unless beaten by more than
                            tie_rtol * (|r| + mu sum |w||v|) of the compared rows */
  double theta;          /* strength threshold; <= 0 picks 0.25 (dim <= 2) / 0.3 */
  int32_t nu1, nu2;      /* pre/post Jacobi sweeps of the V(nu1,nu2) cycle */
  double omega;          /* Jacobi weight */
  int32_t coarse_max;    /* dense direct solve at or below this many unknowns */
  int32_t max_levels;
  int32_t verbose;       /* 1: one line per outer iteration on stderr */
  void* stream;          /* hipStream_t to order work on; NULL = handle's stream */
  double reuse_frac;     /* keep the AMG splitting and interpolation of the last
                            full setup (recomputing only the Galerkin products)
                            while fewer than reuse_frac * n policy entries have
                            changed since; 0 rebuilds the hierarchy every step */
  double forcing;        /* inexact policy iteration: when > 0 each linear solve
                            stops once ||b - A v||_inf <= forcing times the
                            Shapley residual of the previous step (or the
                            lin_rtol/lin_atol test, whichever is looser).
                            0 (default) solves every system to lin_rtol. */
  int32_t smoother;      /* SHAPLEY_SMOOTH_*; default SHAPLEY_SMOOTH_JACOBI */
  int32_t gamma;         /* cycle index of Algorithm MGcycle: 1 = V-cycle
                            (default), 2 = W-cycle (the coarse problem is
                            visited twice per level) */
  int32_t graph;         /* 1 (default): the launches of one refinement cycle
                            are captured once per AMG hierarchy into a HIP
                            graph and replayed; 0: launched one by one.  The
                            results are the same bit for bit. */
} shapley_solve_opts;

/* Per-solve statistics (the paper's table columns, Sec. 6, plus timings). */
typedef struct shapley_stats {
  int32_t outer;             /* k: MAX policy iterations */
  int32_t inner_total;       /* linear systems solved (sum of n_k) */
  int32_t cycles_total;      /* V-cycles over all linear systems */
  int32_t levels;            /* AMG levels of the last hierarchy */
  int32_t converged;         /* 1 if stopped on eps or policy stability */
  int32_t fmg_levels;        /* grids visited (FAMGpi) */
  double residual;           /* final ||F(v) - v||_inf */
  double residual_l2;        /* final discrete L2 norm sqrt(mean((F(v)-v)^2)) */
  double seconds;            /* wall time of the solve (device-resident data) */
  double setup_seconds;      /* AMG setups (host wall time; a numeric refresh
                                does not wait for the device, its device time
                                is then counted in cycle_seconds) */
  double cycle_seconds;      /* refinement + V-cycles */
  double improve_seconds;    /* assembly + improvement sweeps */
  double op_complexity;      /* sum nnz(A_l) / nnz(A_0) of the last hierarchy */
  double grid_complexity;    /* sum n_l / n_0 */
  int32_t inner_per_outer[64]; /* n_k for k = 1..64 */
  int32_t setups_full;       /* AMG setups built from scratch */
  int32_t setups_refresh;    /* numeric refreshes of a kept hierarchy */
  int32_t value_steps;       /* linear systems solved, accuracy re-solves included */
} shapley_stats;

/* Fills *o with the defaults: eps 0, FP64, AMGpi, c_fmg 1e-2, no warm start,
 * max_outer 100000, max_inner 100000, max_cycles 200, lin_rtol 1e-14,
 * lin_atol 0, tie_rtol 1e-12, theta auto, nu1 = nu2 = 2, omega 0.8,
 * coarse_max 64, max_levels 25, verbose 0, stream NULL, reuse_frac 0.5,
 * forcing 0, smoother SHAPLEY_SMOOTH_JACOBI, gamma 1, graph 1. */
void shapley_default_opts(shapley_solve_opts* o);

/* ---------------------------------------------------------------- games */

/* Flags of shapley_game_create. */
#define SHAPLEY_HOST_PTRS 0u    /* every array is a host array */
#define SHAPLEY_DEVICE_PTRS 1u  /* every array (and grid->bvals) is device memory of the
                                   current HIP device, e.g. a PyTorch tensor's storage */

/*
 * Creates a game handle from its transition stencils: the finite game of
 * Sec. 2 (states, action sets A(x) and B(x,a), transition probabilities
 * p(y|x,a,b), rewards r(x,a,b) and discount mu of eq. (eq1)): states
 * X = {0..n-1}, m1 actions for MAX and m2 for MIN at every state (invalid
 * pairs are masked by `valid`).  Row (x, a, b) = (x*m1 + a)*m2 + b holds the
 * sparse row y -> w = p(y|x,a,b) in CSR form and the reward r(x,a,b).
 *   row_ptr  [n*m1*m2 + 1] int64, row_ptr[0] = 0, non-decreasing
 *   col      [row_ptr[end]] int32 in [0, n)
 *   w        [row_ptr[end]] double >= 0, sum of each row <= 1 + 1e-12
 *   r        [n*m1*m2] double, finite
 *   mu       discount in (0, 1]; the systems I - mu W must be non-singular
 *            (mu = 1 with substochastic W, as for the discretised PDEs of
 *            Sec. 3.3, is allowed)
 *   valid    optional [n*m1*m2] uint8 (1 = pair allowed); every state needs a
 *            valid a and every valid a a valid b.  NULL = all valid.
 *   grid     optional geometric description (for FAMGpi), or NULL
 *   flags    SHAPLEY_HOST_PTRS: all arrays are host arrays (checked and
 *            copied on the host);  SHAPLEY_DEVICE_PTRS: all arrays, including
 *            grid->bvals, are device memory of the current device (checked by
 *            a kernel, copied device to device; nothing goes through the
 *            host but row_ptr[n*m1*m2] and the check's result).  Either way
 *            the library copies the arrays and the caller keeps ownership.
 *            Rows whose columns are not ascending are sorted (stable).
 *   stream   hipStream_t for the copies and later work; NULL = a new stream
 *            owned by the handle.  With device pointers, the arrays must be
 *            ready when the call starts (the caller synchronises its own
 *            stream first, or passes that stream here).
 * Errors: SHAPLEY_EINVAL on any violated condition (the game is not
 * created), SHAPLEY_ENOMEM, SHAPLEY_EDEVICE.
 */
int shapley_game_create(shapley_game_t* out, int64_t n, int32_t m1, int32_t m2,
                        const int64_t* row_ptr, const int32_t* col, const double* w,
                        const double* r, double mu, const uint8_t* valid,
                        const shapley_grid* grid, uint32_t flags, void* stream);

/*
 * Builds a hierarchy handle for FAMGpi (Algorithm algo-FAMGPI, Sec. 5.2) from
 * nlev games ordered coarse -> fine, each created with a grid description of
 * the same dimension; step h_l of level l halves (or, for non-nested grids,
 * roughly halves) from one level to the next.  The hierarchy takes ownership
 * of the level handles (do not destroy them separately).  Solving the
 * hierarchy with method SHAPLEY_FAMGPI runs AMGpi on every level with
 * eps_l = c_fmg h_l^2 and transfers (v, alpha, beta) upwards by I and U;
 * results are read from the finest level through the hierarchy handle.
 */
int shapley_game_create_hierarchy(shapley_game_t* out, int32_t nlev, shapley_game_t* levels);

/* Solves the game: the fixed point v of the Shapley operator F of eq. (eq1)
 * (Sec. 2) and optimal pure stationary strategies, by policy iteration with an
 * algebraic-multigrid solve of each policy system (AMGpi, Sec. 5.1: the
 * two-player scheme of Algorithm PIalgo whose inner loop is Algorithm
 * algo-MDP, systems (LSPI) solved by the cycles of Algorithm MGcycle), or, for
 * a hierarchy with method SHAPLEY_FAMGPI, by full multilevel policy iteration
 * (Sec. 5.2, Algorithm algo-FAMGPI).  Warm starts alpha0/beta0/v0 (host
 * arrays) are the arguments (alpha, beta, v) of AMGpi in Algorithm
 * algo-FAMGPI: alpha0 must name an available action (one with a valid b) and
 * (alpha0, beta0) a valid pair at every state, else SHAPLEY_EINVAL before any
 * change.  o may be NULL (defaults); st may be NULL.
 * Errors: SHAPLEY_EINVAL (options, warm start), SHAPLEY_ENOCONV (an iteration
 * limit was hit, or MIN's inner loop was cut by max_inner and MAX has no
 * improvement left while the residual is above eps: the value, strategies and
 * stats of the last step are readable), SHAPLEY_EDEVICE (non-finite values or
 * a HIP error), SHAPLEY_ENOMEM. */
int shapley_solve(shapley_game_t g, const shapley_solve_opts* o, shapley_stats* st);

/* Copies the current value v (n doubles; after a converged solve the fixed
 * point of eq. (eq1), Sec. 2) to v: a host array, or device memory of the
 * handle's device if on_device != 0.  Synchronises the handle's stream.
 * Errors: SHAPLEY_EINVAL (null argument), SHAPLEY_EDEVICE. */
int shapley_get_value(shapley_game_t g, double* v, int32_t on_device);

/* Copies the current pure stationary strategies (Sec. 2): alpha[n], MAX's
 * action at each state, and beta[n], MIN's action at (x, alpha(x)); beta_all
 * (optional, n*m1, row-major by state) receives MIN's lowest-index argmin of
 * the bracket of eq. (eq1) at every a for the current value (the strategy
 * beta(x, a) of Sec. 2 on all of X x A).  Host arrays; any may be NULL.  With
 * the value these form the checkpoint a later solve takes as warm start.
 * Errors: SHAPLEY_EINVAL (null game), SHAPLEY_EDEVICE. */
int shapley_get_policy(shapley_game_t g, int32_t* alpha, int32_t* beta, int32_t* beta_all);

/* Evaluates the Shapley operator F(v) (Sec. 2, eq. (eq1)) at the host vector
 * v[n]: F[n] and the greedy strategies at v, alpha = lowest-index argmax_a of
 * min_b and beta = lowest-index argmin_b at alpha (host arrays, any output
 * may be NULL).  The handle's value and strategies are left unchanged.
 * Errors: SHAPLEY_EINVAL (null argument), SHAPLEY_EDEVICE. */
int shapley_apply_operator(shapley_game_t g, const double* v, double* F, int32_t* alpha,
                           int32_t* beta);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * operator of shapley_apply_operator with device-resident arguments and no
 * allocation of any kind.  v[n] (input), F[n] (optional), alpha[n], beta[n]
 * (required) and res[2] (optional: max_x |F(v) - v| and sum_x (F(v) - v)^2)
 * are device memory of the current device; the work is queued on `stream`
 * (NULL: the handle's stream) and the call returns without synchronising.
 * Its reductions use a fixed device array of the library (16 KB, the same
 * for every game size; one copy per device, kept until the process ends):
 * calls that overlap on one device race, so order them on one stream.  The
 * results equal shapley_apply_operator's bit for bit.  Errors: SHAPLEY_EINVAL
 * (null handle, v, alpha or beta), SHAPLEY_EDEVICE. */
int shapley_apply_operator_noalloc(shapley_game_t g, const double* v, double* F, int32_t* alpha, int32_t* beta,
                                   double* res, void* stream);

/* n = |X|, m1 and m2 (Sec. 2) of a handle (the finest level for
 * hierarchies).  Errors: SHAPLEY_EINVAL (null game). */
int shapley_game_info(shapley_game_t g, int64_t* n, int32_t* m1, int32_t* m2);

/* Device bytes held by the handle (transitions, rewards, pattern, value and
 * strategies; the solver's workspace is not counted).  The request loop's
 * HBM budget admission builds on it.  Errors: SHAPLEY_EINVAL. */
int shapley_game_bytes(shapley_game_t g, size_t* bytes);

/* Lanes per sparse row in the V-cycle's relaxation, residual and restriction
 * kernels (Sec. 4.3, the multigrid cycle): 0 (default) lets the library time
 * 1, 2 and 4 lanes on each large level at its first setup and keep the
 * fastest per size class (levels under 2^18 entries take a rule on the
 * average row length); 1, 2 or 4 forces that count for every level of later
 * setups.  Row sums are formed in the same order for every count, so results
 * do not depend on this setting.  Process-wide.  Errors: SHAPLEY_EINVAL for
 * any other value. */
int shapley_tune_lanes(int32_t lanes);

/* Kernel choice of the row-wise Galerkin product A_{l+1} = R A_l P (Sec. 4.3)
 * on large levels: -1 (default) lets the library choose per product from the
 * level's average row length; 0 forces the wavefront-per-row kernel alone;
 * 1 first runs a thread-per-row kernel and 4 a four-lanes-per-row kernel,
 * each taking the rows whose columns fit it and handing the others to the
 * wavefront kernel.  Every kernel sums each entry's products in the same
 * order, so results do not depend on this setting.  Process-wide; applies
 * to later setups and refreshes.  Errors: SHAPLEY_EINVAL for any other
 * value. */
int shapley_tune_galerkin(int32_t kernel);

/* Kernel choice of the extended+i interpolation of coarse levels (the
 * prolongation P of Sec. 4.3): 4 first runs a four-lanes-per-row kernel that
 * takes the rows whose sets fit it and hands the others to the wavefront-per-
 * row kernel; 0 forces the wavefront kernel alone; -1 (default) takes the
 * four-lane kernel on levels of 2^16 rows or more whose rows average at most
 * 24 entries.  Both
 * form every weight with the same operations in the same order, so results
 * do not depend on this setting.  Process-wide; applies to later setups.
 * Errors: SHAPLEY_EINVAL for any other value. */
int shapley_tune_interp(int32_t kernel);

/* Storage of the matrices read by the relaxation sweeps and residuals of the
 * multigrid cycle (Algorithm MGcycle, Sec. 4.3) and the FP64 residual of the
 * refinement: -1 (default) stores the finest level as a stencil -- value
 * slots by row, columns from a few per-game offsets -- when every game of
 * the solve has a level-0 pattern of at most 8 distinct offsets col - x and
 * rows of at most 8 entries (grid games) and the relaxation is not C/F, and
 * gives the other levels' columns as 16-bit offsets from the row where all
 * fit; 0 keeps CSR with 32-bit columns everywhere.  Every form sums each
 * row's entries in the same order, so results do not depend on this
 * setting.  Process-wide; applies to later solves.  Errors: SHAPLEY_EINVAL
 * for any other value. */
int shapley_tune_stencil(int32_t mode);

/* Kernel of the exact solve on the coarsest level of the multigrid cycle
 * (Algorithm MGcycle, Sec. 4.3), whose blocks are inverted once per setup:
 * -1 (default) inverts blocks of at most 64 unknowns with the FP64 matrix
 * cores (a blocked Gauss-Jordan sweep over panels of 16 columns with partial
 * pivoting); 0 takes the register Gauss-Jordan kernel with partial pivoting
 * for them.  Larger blocks always take the Gauss-Jordan kernels.  The two
 * differ in rounding order only (results agree to a few units in the last
 * place times the block's condition number).  Process-wide; applies to later
 * setups.  Errors: SHAPLEY_EINVAL for any other value. */
int shapley_tune_dense(int32_t kernel);

/* The coarsest-level inverse of Algorithm MGcycle (Sec. 4.3) on given dense
 * blocks, with the kernels the solver uses (shapley_tune_dense selects the
 * one for blocks of at most 64 unknowns): a testing and inspection aid.
 *   a:     count blocks back to back, block g of sizes[g] x sizes[g] entries,
 *          row-major, finite (host, read only);
 *   sizes: count block sizes in 1 .. 1024 (host);
 *   inv:   receives the inverses in the layout of a (host, caller-owned).
 * Runs on the null stream and synchronises it.  Errors: SHAPLEY_EINVAL (null
 * argument, count < 0, a size out of range, a non-finite entry),
 * SHAPLEY_EDEVICE when a block is singular (no nonzero pivot left),
 * SHAPLEY_ENOMEM. */
int shapley_coarse_inverse(const double* a, const int32_t* sizes, int32_t count, double* inv);

/* Testing aid for the error paths (no passage of the paper: library
 * robustness).  after > 0: the after-th device allocation made by the library
 * from now on fails as if the device were out of memory, so that the call
 * making it returns SHAPLEY_ENOMEM; 0 disarms.  Handles stay usable after
 * such a failure (a later call allocates again).  Process-wide.  Errors:
 * SHAPLEY_EINVAL for after < 0. */
int shapley_debug_fail_alloc(int64_t after);

/* Inspection of the algebraic multigrid hierarchy (Sec. 4.3) built by the
 * last shapley_solve of g, run alone on the handle's own stream (opts.stream
 * NULL; for a hierarchy handle, the finest grid's).  Level 0 is the operator
 * I - mu P of the last policy pair the hierarchy was built or refreshed from;
 * level l+1 is the Galerkin product P_l^T A_l P_l.
 *   info: levels (count), pw (slots per row of P), n, nnz (of A_level) and nc
 *         (rows of level+1, 0 on the last level).
 *   rp[n+1], ci[nnz], a[nnz]: A_level in CSR, columns sorted within a row.
 *   pc[n*pw], pv[n*pw]: P_level by rows (column index into level+1, -1 for
 *         an empty slot), written only when nc > 0.
 * Host arrays owned by the caller, each may be NULL (call first with NULL
 * arrays for the sizes).  Synchronises the handle's stream.  Errors:
 * SHAPLEY_EINVAL when no such hierarchy is held (another solve ran on the
 * stream since, or the game was solved in a batch) or level is out of
 * range. */
typedef struct shapley_level_info {
  int32_t levels;
  int32_t pw;
  int64_t n;
  int64_t nnz;
  int64_t nc;
} shapley_level_info;
int shapley_hierarchy_level(shapley_game_t g, int32_t level, shapley_level_info* info, int32_t* rp, int32_t* ci,
                            double* a, int32_t* pc, double* pv);

/* Releases the handle (a hierarchy releases its levels) and the device
 * memory it holds; NULL is ignored.  The handle must not be in use by a
 * solve or by a server ticket that has not completed. */
void shapley_game_destroy(shapley_game_t g);

/* ---------------------------------------------------------------- batch */

/*
 * Solves `count` independent games in lock-step: every V-cycle level of all
 * games is processed by one launch per kernel (block-diagonal merged levels),
 * games that converge leave the active set.  Results of each game equal those
 * of solving it alone within the linear-solve tolerance.  stats (optional)
 * receives count entries.  FAMGpi hierarchies are not accepted here.
 */
int shapley_solve_batch(shapley_game_t* games, int32_t count, const shapley_solve_opts* o,
                        shapley_stats* stats);

/* ---------------------------------------------------------------- server */

/*
 * A request loop with continuous batching (the serving mode of the solver; the
 * solve of each request is that of shapley_solve, AMGpi of Sec. 5.1 or FAMGpi
 * of Sec. 5.2): submitted games (or hierarchies) are admitted in FIFO order
 * while their estimated device footprint fits the budget.  Requests admitted
 * in the same step with equal engine options (precision, AMG and cycle
 * options, tie_rtol) form a cohort: one lock-step engine with merged
 * launches and an AMG hierarchy kept on the device until the cohort's last
 * member leaves; members that converge leave without a rebuild.  Cohorts
 * run concurrently on streams of their own (one host thread each), so
 * requests admitted while others run overlap with them on the device.  An
 * FAMGpi request moves to a new cohort at each finer grid.  At 16 cohorts,
 * new requests join the compatible cohort with the fewest running unknowns.
 *   hbm_budget  bytes of device memory the server may hold for requests
 *   stream      NULL: streams owned by the server (cohorts concurrent); a
 *               caller's hipStream_t: every cohort on it, one after another
 * Errors: SHAPLEY_EINVAL (null out, zero budget), SHAPLEY_EDEVICE.
 */
int shapley_server_create(shapley_server_t* out, size_t hbm_budget, void* stream);
/* Queues g (ownership stays with the caller; do not use or destroy g until
 * its ticket completes).  Options and warm starts are checked here as in
 * shapley_solve.  Thread-safe.  Errors: SHAPLEY_EINVAL, SHAPLEY_ENOMEM when
 * the request's footprint alone exceeds the whole budget. */
int shapley_server_submit(shapley_server_t srv, shapley_game_t g, const shapley_solve_opts* o,
                          uint64_t* ticket);
/* Runs scheduling steps until the ticket completes or `max_steps` steps pass
 * (max_steps <= 0: until complete).  Returns SHAPLEY_EAGAIN if not complete. */
int shapley_server_wait(shapley_server_t srv, uint64_t ticket, int32_t max_steps,
                        shapley_stats* st);
/* Non-blocking: SHAPLEY_OK if the ticket completed (stats filled), else EAGAIN. */
int shapley_server_poll(shapley_server_t srv, uint64_t ticket, shapley_stats* st);
/* Runs one scheduling step (admission + one PI step of all active requests).
 * *active receives the number of requests not yet completed (on the device
 * or queued).  A request whose solve fails completes with the error code of
 * the failure (poll/wait return it and shapley_last_error its message); the
 * other members of its cohort complete with the same code. */
int shapley_server_step(shapley_server_t srv, int32_t* active);
/* Occupancy of the request loop. */
typedef struct shapley_server_stats {
  int32_t queued;        /* submitted, not admitted */
  int32_t active;        /* admitted, not completed */
  int32_t cohorts;       /* engines with running members */
  int32_t reserved;
  size_t budget_used;    /* estimated device bytes of the active requests */
  size_t budget;
} shapley_server_stats;
int shapley_server_info(shapley_server_t srv, shapley_server_stats* st);
void shapley_server_destroy(shapley_server_t srv);

/* ---------------------------------------------------------------- probe */

/* Kernel families of the timing probe. */
enum {
  SHAPLEY_PROBE_SMOOTH = 0,   /* weighted-Jacobi relaxation, all AMG levels */
  SHAPLEY_PROBE_RESID64 = 1,  /* FP64 residual of the iterative refinement */
  SHAPLEY_PROBE_IMPROVE = 2,  /* policy improvement + Shapley residual sweep */
  SHAPLEY_PROBE_RESID = 3,    /* cycle residual, all levels */
  SHAPLEY_PROBE_RESTRICT = 4, /* restriction R r */
  SHAPLEY_PROBE_PROLONG = 5,  /* prolongation + correction u += P e */
  SHAPLEY_PROBE_RAP = 6,      /* Galerkin product (setup) */
  SHAPLEY_PROBE_INTERP = 7,   /* interpolation (setup) */
  SHAPLEY_PROBE_TAIL = 8      /* coarse levels of a game's V-cycle in one workgroup */
};

/* Enables (on != 0) or disables the timing probe of one kernel family and
 * resets its totals.  While enabled, every launch of the family is bracketed
 * by HIP events on its stream (this adds a little host overhead). */
int shapley_probe_enable(int32_t family, int32_t on);

/* Totals since the probe was enabled: launches, summed device time between
 * the bracketing events (ms) and summed algorithmic bytes of the launches
 * (bytes the kernel must read and write at minimum, each value once).
 * Synchronises with the recorded events. */
int shapley_probe_read(int32_t family, int64_t* launches, double* total_ms, double* total_bytes);

/* The same totals over the largest launches only: those whose algorithmic
 * bytes are at least frac (0 < frac <= 1) times the largest launch's since
 * the probe was enabled.  A family's launches on the finest level of the
 * largest game are its largest, so frac = 0.5 isolates them (the next level
 * of a 2-D grid holds about a quarter of the rows).  Synchronises like
 * shapley_probe_read.  SHAPLEY_EINVAL on a bad family or frac;
 * SHAPLEY_ENOMEM when more than 2^20 launches were probed since enabling
 * (per-launch records are kept up to that many). */
int shapley_probe_read_large(int32_t family, double frac, int64_t* launches, double* total_ms,
                             double* total_bytes);

#ifdef __cplusplus
}
#endif
#endif /* SHAPLEY_H */
