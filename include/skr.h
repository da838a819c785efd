/*
 * skr.h -- C ABI of the MI355X (gfx950) Sorting Krylov Recycling library (libskr.so).
 *
 * The library orders a batch of related sparse linear systems A_i x_i = b_i (Eq. 1) by the
 * greedy nearest-neighbour sort of Alg. 1 (Sec. 4.1), and solves them in that order with
 * GCRO-DR (Alg. 2, App. B.2), carrying the recycled subspace U_k from each system to the next
 * (App. B.1). Plain restarted GMRES(m) is the same call with k = 0 (Sec. 4.2).
 *
 * Conventions for every entry point
 *  - Pointers named *_dev are device pointers on the context's device; pointers named *_host are
 *    host pointers. The caller owns all of them: the library never frees caller memory and reads
 *    or writes it only during the call.
 *  - All work is enqueued on the stream given to skr_ctx_create. Calls return after their
 *    results are final (they synchronise that stream), so inputs may be reused at once.
 *  - Floating point is IEEE FP64; indices are int32, orderings int64.
 *  - Return value: 0 = success, < 0 = error (nothing further promised, skr_last_error() gives a
 *    message), > 0 = completed with a warning.
 *  - A context is not thread-safe: one host thread at a time per context.
 */
#ifndef SKR_H
#define SKR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define SKR_OK                 0
#define SKR_EINVAL            (-1)   /* bad sizes or options (e.g. k < 0, m <= k, rtol <= 0)   */
#define SKR_ENOMEM            (-2)   /* device workspace could not be allocated                */
#define SKR_EHIP              (-3)   /* HIP runtime failure                                    */
#define SKR_ENONFINITE        (-4)   /* NaN or Inf in an input where none is allowed           */
#define SKR_WARN_NOTCONVERGED   1    /* at least one system stopped at maxit                   */
#define SKR_PENDING             2    /* skr_poll: the ticket's system is not solved yet        */

/* per-system status (skr_result.status) */
#define SKR_CONVERGED   0   /* ||b - A x|| <= rtol ||b||                                        */
#define SKR_MAXIT       1   /* stopped after maxit Arnoldi steps without meeting the tolerance  */
#define SKR_BREAKDOWN   2   /* converged through a happy breakdown (invariant Krylov subspace)  */
#define SKR_NONFINITE   3   /* b or A holds NaN/Inf; x is set to zero, nothing is recycled      */

/* operator kinds (skr_op.kind) */
#define SKR_OP_CSR      0   /* general sparse matrix, CSR                                        */
#define SKR_OP_STENCIL5 1   /* matrix-free 2-D 5-point operator built from face coefficients   */
#define SKR_OP_STENCIL7 2   /* matrix-free 3-D 7-point operator built from face coefficients   */

typedef struct skr_ctx skr_ctx;

/*
 * One system matrix A (n x n). Device pointers, caller-owned.
 *  CSR:      rowptr[n+1], colind[nnz] (0-based), values[nnz]; rows need not be sorted.
 *  STENCIL5: unknowns on an nx-by-ny grid, unknown (i, j) (row i < ny, column j < nx) at index
 *            i*nx + j (row-major as in the worked example of Sec. 3.1 / App. A);
 *            ax[ny*(nx+1)]: ax[i*(nx+1) + j] is the coefficient on the face between columns
 *            j-1 and j of row i (j = 0 and j = nx are the Dirichlet boundary faces);
 *            ay[(ny+1)*nx]: ay[i*nx + j] is the face between rows i-1 and i of column j.
 *            (A x)_ij = inv_h2 * ( sum of the 4 faces * x_ij - sum over interior neighbours of
 *            face * x_neighbour ), i.e. -div(a grad u) with zero Dirichlet data.
 *  STENCIL7: the same in 3-D on an nx-by-ny-by-nz grid, unknown (x, y, z) at index
 *            x + nx*(y + ny*z); ax[nz*ny*(nx+1)]: ax[(z*ny + y)*(nx+1) + x] is the face between x-1
 *            and x; ay[nz*(ny+1)*nx]: ay[(z*(ny+1) + y)*nx + x] the face between y-1 and y;
 *            az[(nz+1)*ny*nx]: az[(z*ny + y)*nx + x] the face between z-1 and z (index 0 and the
 *            last index are the Dirichlet boundary faces). Uses nz and az; nx, ny, inv_h2, ax, ay as
 *            for STENCIL5.
 */
typedef struct {
    int32_t kind;
    int32_t n;
    int32_t nnz;
    const int32_t* rowptr;
    const int32_t* colind;
    const double* values;
    int32_t nx, ny;
    double inv_h2;
    const double* ax;
    const double* ay;
    int32_t nz;             /* STENCIL7 only */
    const double* az;       /* STENCIL7 only */
} skr_op;

/* Solver options. m: maximum subspace size per cycle (1..86); k: recycled vectors (0 = GMRES(m),
 * k < m, k <= 32); rtol: relative residual target; maxit: maximum Arnoldi steps per system;
 * flags: 0 or a combination of SKR_FLAG_PROFILE, SKR_FLAG_FOLD, SKR_FLAG_MIXED and SKR_FLAG_CONTINUE. */
#define SKR_FLAG_PROFILE 1u   /* time every 16th Arnoldi step's kernels with hipEvents (see skr_profile_get) */
#define SKR_FLAG_FOLD    2u   /* fold the per-workgroup partials of every grid reduction into 64 rows
                                 before they are re-summed; done anyway above 256 workgroups
                                 (n > 65,536), where it keeps the reduction cost linear in n */
#define SKR_FLAG_MIXED   4u   /* mixed precision: the Arnoldi vectors and the recycle pair C_k, U_k
                                 are stored in FP32 (round to nearest even), and the inner cycle's
                                 products with A (the Arnoldi steps and the start-up A*Y) use the
                                 operator's values (CSR values, stencil faces) rounded to FP32,
                                 halving the bytes the Arnoldi steps stream; every sum and product is
                                 formed in FP64, and x, r and the small dense problems stay FP64. Each
                                 cycle after the first starts from the true residual r = b - A x with
                                 the FP64 operator, projected onto range(C) (x += U C^T r,
                                 r -= C C^T r): iterative refinement with one cycle as the inner
                                 correction. relres_true is the FP64 residual of the FP64 solution,
                                 so rtol keeps its meaning. An extension of the paper's method
                                 (Alg. 2 is stated in exact arithmetic). */
#define SKR_FLAG_CONTINUE 8u  /* skr_solve_sequence: the first system starts from the recycle space
                                 the context carries (left by the previous skr_solve_sequence on it,
                                 or set with skr_recycle_set) instead of none; it must belong to the
                                 same n, m, k and SKR_FLAG_MIXED setting, else SKR_EINVAL */

typedef struct {
    int32_t m;
    int32_t k;
    double rtol;
    int64_t maxit;
    uint32_t flags;
} skr_opts;

/* Per-system result, written at the system's original index. */
typedef struct {
    int32_t status;        /* SKR_CONVERGED, SKR_MAXIT, SKR_BREAKDOWN or SKR_NONFINITE            */
    int32_t cycles;        /* Arnoldi cycles run                                                  */
    int32_t k_start;       /* recycled vectors kept by the start-up QR of A*Y (0 without recycling)*/
    int32_t rank_dropped;  /* recycled vectors dropped as numerically dependent at start-up       */
    int64_t iters;         /* Arnoldi steps                                                       */
    int64_t spmv;          /* products with A: Arnoldi, start-up A*Y columns, true residuals      */
    double relres_true;    /* ||b - A x|| / ||b||, computed on the device at exit                 */
    double relres_est;     /* least-squares residual estimate / ||b|| at exit                     */
    double seconds;        /* host wall-clock time of the system's solve (start-up to exit test;   */
                           /* the call waits for the device at the end of every system)            */
} skr_result;

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t, NULL for
 * the default stream).
 * arena_dev, arena_bytes: a caller-owned device buffer (e.g. a torch tensor) that the context
 * sub-allocates for all its device memory: the workspace of each solve (one block of
 * skr_workspace_bytes), the carried recycle space, the sort's distance matrix and outputs, the FP32
 * operator copy of the mixed mode (4 bytes per CSR value or stencil face), and in serving every
 * chain's workspace, resident recycle space and parameter tail (skr_workspace_bytes + 8p bytes,
 * rounded up to 256). The buffer must stay valid until skr_ctx_destroy; the library never frees it.
 * When a request does not fit, the call fails with SKR_ENOMEM (serving defers the admission
 * instead, retiring idle chains first, Sec. 4.1 / App. E chains). Both NULL / 0: the library
 * allocates its own memory. Only the serving runtime's small staging buffers (distance partials and
 * deferred parameter copies) are allocated outside the arena.
 * Returns SKR_EINVAL for a bad device or a half-given arena, SKR_EHIP on runtime failure. */
int skr_ctx_create(int device, void* hip_stream, void* arena_dev, size_t arena_bytes, skr_ctx** out);

/* Device bytes of the workspace a context allocates for solves of size n with GCRO-DR(m, k) (basis
 * [C V], U and A C, work vectors, reduction partials, small dense state), as one block; the same
 * for both storage modes (flags: SKR_FLAG_* of the solve). A serving chain adds p doubles for its
 * parameter tail, rounded up to 256 bytes. Returns 0 for sizes a solve would reject (n < 1 or
 * n >= 2^31, m outside [1, 86], k < 0, k >= m, k > 32). */
size_t skr_workspace_bytes(int64_t n, int32_t m, int32_t k, uint32_t flags);

/* Free the context and its workspace (waits for its stream). NULL is accepted. */
int skr_ctx_destroy(skr_ctx* ctx);

/* Message for the last failing call on this host thread ("" if none). */
const char* skr_last_error(void);

/* Library version string. */
const char* skr_version(void);

/*
 * Greedy nearest-neighbour order of N systems (Alg. 1, Sec. 4.1).
 *  params_dev: N x p row-major FP64 parameter matrices (row i = vec(P^(i))).
 *  start: index of the first system (Alg. 1 starts at the first system: pass 0).
 *  order_host: out, N int64, a permutation of 0..N-1 with order_host[0] = start.
 *  step_d2_host: optional out (NULL to skip), N FP64, squared distance of each step (entry 0 = 0).
 * Each step appends the unvisited system with the smallest squared Frobenius distance
 * sum_p (P_cur[p] - P_j[p])^2 to the system appended last; the sum of the squares of the FP64
 * differences is accumulated in double-double and rounded once, ties go to the lowest index,
 * NaN/Inf distances are never preferred. Errors: SKR_EINVAL (N < 0, p < 1 with N > 0, start out
 * of range), SKR_ENOMEM.
 */
int skr_sort(skr_ctx* ctx, const double* params_dev, int64_t N, int64_t p, int64_t start,
             int64_t* order_host, double* step_d2_host);

/*
 * skr_sort without any device allocation, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc). Same arguments, results
 * (bit for bit) and errors as skr_sort, for N <= 512 systems and any p. The distance matrix, slice
 * partials and outputs live in one library-owned static device array of 16 MiB per GPU, held until
 * the process ends; the caller passes only the inputs and outputs. Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (several host threads or streams) race: serialise
 * them. Errors: those of skr_sort, SKR_EINVAL for N > 512, SKR_EHIP if the array could not be
 * located on the device.
 */
int skr_sort_noalloc(skr_ctx* ctx, const double* params_dev, int64_t N, int64_t p, int64_t start,
                     int64_t* order_host, double* step_d2_host);

/*
 * Solve A_i x_i = b_i for i = order[0], order[1], ... (Eq. 1) with GCRO-DR(m, k) (Alg. 2),
 * x0 = 0, carrying U_k from each solved system to the next (App. B.1).
 *  ops:    host array of N operators (device data), indexed by original system index;
 *          all must have the same n.
 *  b_dev:  host array of N device pointers to right-hand sides (n FP64 each).
 *  x_dev:  host array of N device pointers, out, solutions (n FP64 each).
 *  order:  host array of N int64 (a permutation), or NULL for 0..N-1.
 *  results_host: out, N entries at the original indices.
 * Every cycle that follows another starts from a residual projected onto the orthogonal complement
 * of range(C_k) (x += U_k C_k^T r, r -= C_k C_k^T r, the start-up step of App. B.1): zero in exact
 * arithmetic, it keeps the cycle's first Krylov vector orthogonal to C_k in floating point, and so
 * C_k orthonormal and the solve stable down to the attainable accuracy. When the least-squares
 * estimate meets rtol but the true residual does not, the solve goes on from the projected true
 * residual. For the cycle-end eigenproblem the symmetric eigen stage is used only for an exactly
 * symmetric operator (the stencil kinds, or a CSR matrix that passes an exact check at the system
 * start); any other operator takes the general stage.
 * Returns SKR_OK, SKR_WARN_NOTCONVERGED if some system hit maxit, or an error
 * (SKR_EINVAL, SKR_ENOMEM, SKR_EHIP). A system with NaN/Inf in b or A gets status
 * SKR_NONFINITE and x = 0; the sequence goes on.
 */
int skr_solve_sequence(skr_ctx* ctx, const skr_op* ops, const double* const* b_dev,
                       double* const* x_dev, int64_t N, const int64_t* order,
                       const skr_opts* opts, skr_result* results_host);

/*
 * Several chains of one sorted order advanced together (the data-parallel split of App. E: the
 * sorted sequence cut into contiguous chains, one per worker, each recycling along its own part).
 * Chain c solves order[chain_start[c]] .. order[chain_start[c+1] - 1] exactly as
 * skr_solve_sequence would on a context of its own (x0 = 0; no recycle space at its first system,
 * or with SKR_FLAG_CONTINUE the one chain c left at the end of the previous skr_solve_chains call
 * on this context), and the results and solutions equal that call's bit for bit. All chains share the context's stream:
 * every kernel launch covers the chains that take part in that phase (one grid row per chain), so
 * C chains cost about the launches of one, which is what raises the throughput of small systems.
 *  C:            number of chains, >= 1.
 *  chain_start:  host array of C + 1 int64, chain_start[0] = 0, chain_start[C] = N, non-decreasing
 *                (an empty chain is allowed).
 *  ops, b_dev, x_dev, N, order, opts, results_host: as for skr_solve_sequence; all operators of
 *                one kind and size. With SKR_FLAG_CONTINUE, C and (n, m, k, precision) must be
 *                those of the previous call on this context (else SKR_EINVAL); a chain may then be
 *                given one system per call, e.g. one time step of C time-stepping chains whose
 *                right-hand sides depend on the previous solutions.
 * Memory: one workspace per chain (C times skr_workspace_bytes) plus small tables, taken from the
 * context's arena when it has one, else allocated; they stay with the context (holding each
 * chain's recycle space) until a call with fewer chains or skr_ctx_destroy. The context's own
 * recycle space (skr_recycle_get) is not touched. Returns as skr_solve_sequence.
 */
int skr_solve_chains(skr_ctx* ctx, int32_t C, const int64_t* chain_start, const skr_op* ops,
                     const double* const* b_dev, double* const* x_dev, int64_t N, const int64_t* order,
                     const skr_opts* opts, skr_result* results_host);

/*
 * Checkpoint and resume of a chain. After skr_solve_sequence the context carries the recycle space
 * U_k that the next system of the chain would start from (the Y~_k handed from system to system,
 * App. B.1; Alg. 2 start-up). With the order and the index of the next system it is the whole
 * state of the chain: every other quantity of a solve is rebuilt from A, b and U_k. A chain split
 * into several skr_solve_sequence calls, the later ones with SKR_FLAG_CONTINUE after
 * skr_recycle_get / skr_recycle_set (also across contexts or processes), gives results identical
 * bit for bit to the uninterrupted call.
 *
 * skr_recycle_get: *k_out receives the number of carried columns (0 after GMRES, k = 0, or when no
 * recycle space was formed). If U_dev is not NULL, U_dev (device, FP64, column-major, leading
 * dimension ld >= n) receives the n x *k_out block; with SKR_FLAG_MIXED the stored FP32 values are
 * widened exactly. Errors: SKR_EINVAL (NULL ctx or k_out, no completed solve on this context,
 * ld < n).
 *
 * skr_recycle_set: makes U_dev (device, FP64, n x kcols, column-major, leading dimension ld) the
 * recycle space the next skr_solve_sequence with SKR_FLAG_CONTINUE and these options starts from.
 * The workspace is sized for (n, opts->m, opts->k) as by a solve; with SKR_FLAG_MIXED the values are
 * rounded to FP32 (nearest even). The caller keeps ownership of U_dev. Errors: SKR_EINVAL (bad
 * options, n < 1, kcols outside [0, opts->k], NULL U_dev or ld < n with kcols > 0), SKR_ENOMEM.
 */
int skr_recycle_get(skr_ctx* ctx, int32_t* k_out, double* U_dev, int64_t ld);
int skr_recycle_set(skr_ctx* ctx, const skr_opts* opts, int64_t n, int32_t kcols, const double* U_dev,
                    int64_t ld);

/* y_dev = A x_dev for one operator (the sparse product of the Arnoldi step; Eq. 3). */
int skr_spmv(skr_ctx* ctx, const skr_op* op, const double* x_dev, double* y_dev);

/* Launch the SpMV kernel `repeats` times back to back between two hipEvents on the context's stream
 * and return the mean duration of one launch in *ms_per_launch (host pointer). Errors: SKR_EINVAL. */
int skr_spmv_repeat(skr_ctx* ctx, const skr_op* op, const double* x_dev, double* y_dev, int32_t repeats,
                    double* ms_per_launch);

/* Kernel statistics gathered by solves run with SKR_FLAG_PROFILE. Each Arnoldi step is three
 * kernels: A (v_j = w / h, w = A v_j, first projection Q^T w), B (w -= Q h1, second projection
 * Q^T w) and C (w -= Q h2, ||w||, Givens update), with Q = [C_k, V_j] (Eq. 6, CGS2). Sampled launches
 * are timed with hipEvents on the context's stream; bytes are the algorithmic HBM bytes of those
 * launches (matrix and basis columns read once, vectors read/written once). */
typedef struct {
    int64_t launches;   /* timed launches                                   */
    double ms;          /* summed duration of the timed launches           */
    double bytes;       /* summed algorithmic bytes of the timed launches  */
} skr_kernel_stat;

typedef struct {
    skr_kernel_stat step_a, step_b, step_c;
    int64_t steps;        /* Arnoldi steps run by profiled solves                 */
    int64_t cycles;       /* Arnoldi cycles run by profiled solves                */
    double step_bytes;    /* algorithmic bytes of all those steps (A + B + C)     */
    /* Cycle ends that formed a recycle space (Alg. 2, harmonic Ritz step), counted for every solve
     * on the context (profiled or not), by the eigen stage that formed it: the symmetric stage
     * (taken only when the operator is exactly symmetric: a stencil kind, or a CSR matrix that
     * passes an exact check at the system start) or the general one. */
    int64_t eig_symmetric;
    int64_t eig_general;
} skr_profile;

/* Copy the statistics accumulated since the last reset into *out (host pointer). */
int skr_profile_get(skr_ctx* ctx, skr_profile* out);

/* Clear the accumulated statistics. */
int skr_profile_reset(skr_ctx* ctx);

/* ---------------------------------------------------------------------------------------------
 * Serving: systems arrive one at a time (continuous batching).
 *
 * The sorted-sequence idea (Sec. 4.1, Alg. 1: each system is solved after its nearest neighbour;
 * App. E: contiguous slices of the sorted order are independent chains) applied online. A submitted
 * system joins the chain whose most recently admitted system is nearest to it in d2 (the exact
 * squared distance of the parameter vectors, as in skr_sort; ties to the lower chain id), among the
 * chains of the same shape (n, p, m, k and SKR_FLAG_MIXED). It starts a new chain when no chain of
 * its shape exists, or when d2 > split_d2_rel * ||params||^2 and a chain can be added without
 * retiring one. With max_chain_systems > 0 a chain that has taken that many systems is full: only
 * chains that are not full are candidates, and when all of a shape are full the system starts a
 * new chain if one can be added without retiring one (else it joins the nearest full chain) - the
 * online form of cutting a sorted sequence into contiguous batches, one per worker (App. E), so
 * that one shape's systems spread over several chains and workers. Each chain
 * owns a HIP stream, a workspace and its recycle space, which stays resident in device memory
 * between systems; its systems are solved in admission order, each starting from the recycle space
 * the previous one left (Alg. 2), so a result depends only on the chain's history, never on timing
 * or on the other chains. Host worker threads drive up to `workers` chains at once.
 *
 * Admission is by workspace bytes: a new chain is created only while the chains' workspaces fit in
 * arena_bytes (0: no limit) and fewer than max_chains exist. For a shape that has no chain, idle
 * chains (nothing queued or running) are retired, least recently used first, to make room; if
 * none is idle the system waits (deferred admission) and is assigned when room frees, as are the
 * systems submitted after it. Only retirement and deferral depend on timing. A system whose
 * workspace alone exceeds arena_bytes is refused with SKR_ENOMEM.
 * --------------------------------------------------------------------------------------------- */
typedef struct {
    int32_t max_chains;     /* chains held at once (>= 1)                                       */
    int32_t workers;        /* host threads driving chains concurrently (>= 1)                  */
    uint64_t arena_bytes;   /* device bytes all chain workspaces may take together, 0 = no limit */
    double split_d2_rel;    /* start a new chain above this relative d2 (INFINITY: never)        */
    int32_t max_chain_systems;  /* systems a chain takes before it is full (0: no limit)          */
    int32_t pad0;
} skr_serve_opts;

typedef struct {
    int64_t submitted, completed;
    int32_t chains_live, chains_created, chains_retired, deferred;
    uint64_t bytes_in_use;  /* device bytes of the live chains' workspaces */
} skr_serve_stats;

/* Start serving on the context's device (the context's stream is used for the distance products
 * at submission). SKR_EINVAL if already started or the options are out of range. */
int skr_serve_start(skr_ctx* ctx, const skr_serve_opts* opts);

/* Submit A x = b with parameter vector params_dev[p] (device, FP64; copied before return, the
 * caller may reuse it). op, b_dev and x_dev are caller-owned device memory that must stay valid
 * until the ticket is reported done; x_dev receives the solution. opts as for skr_solve_sequence
 * (all systems of a chain share m, k and the SKR_FLAG_MIXED setting). *ticket receives an id > 0.
 * Errors: SKR_EINVAL (not serving, bad arguments), SKR_ENOMEM (workspace larger than the arena),
 * SKR_EHIP. Thread-safe. */
int skr_submit(skr_ctx* ctx, const skr_op* op, const double* params_dev, int64_t p, const double* b_dev,
               double* x_dev, const skr_opts* opts, uint64_t* ticket);

/* SKR_PENDING while the system is queued or running; when it is done, writes the result (host)
 * and returns SKR_OK, or the error code of a failed solve (skr_last_error() has the message).
 * A ticket is collected by the first call that reports it done; later calls return SKR_EINVAL. */
int skr_poll(skr_ctx* ctx, uint64_t ticket, skr_result* out);

/* skr_poll that blocks until the ticket is done. */
int skr_wait(skr_ctx* ctx, uint64_t ticket, skr_result* out);

/* The chain a ticket was assigned to and its position in that chain (0 = the chain's first
 * system), or -1 / -1 while its admission is deferred. Valid until the ticket is collected. */
int skr_ticket_chain(skr_ctx* ctx, uint64_t ticket, int32_t* chain, int64_t* position);

/* Counters of the serving runtime (host pointer). */
int skr_serve_stats_get(skr_ctx* ctx, skr_serve_stats* out);

/* Finish every submitted system, then free the chains and stop the workers. Uncollected results
 * are dropped. Called by skr_ctx_destroy if serving is still on. */
int skr_serve_stop(skr_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SKR_H */
