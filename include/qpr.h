/*
 * qpr.h -- C ABI of libqpr, an MI355X (gfx950) solver for the steady state of
 * quantum PageRank (Tang, He, Shi, Zhu, Lee, Wang, Jin, "TensorFlow Solver for
 * Quantum PageRank in Large-Scale Networks", arXiv:2003.04930).
 *
 * The solver integrates the quantum-stochastic-walk Lindblad equation (Eq. (1),
 * Supplementary Eq. (S7))
 *
 *   d rho/dt = L(rho) = -i (1-omega) [H, rho] + omega D_G(rho),
 *   D_G(rho) = sum_ij ( L_ij rho L_ij^dag - 1/2 {L_ij^dag L_ij, rho} ),
 *   L_ij     = sqrt(G_ij) |i><j|,
 *
 * with the classical four-stage Runge-Kutta method or the adaptive Fehlberg
 * 4(5) method (Supplementary Note 2) until ||L(rho)||_F < tol.  The
 * N^2 x N^2 Liouvillian of Eq. (2) is never formed: the commutator is one
 * real product X = H_off [Re rho | Im rho] (dense on the matrix cores, or
 * gathers through the sparsity pattern of H_off) and
 * [H, rho] = X - X^dag + [diag(h), rho]; the jump sum
 * collapses to diag(G p) - 1/2 (d_a + d_b) rho_ab with p = diag(rho) and
 * d_j = sum_i G_ij.
 *
 * Conventions (every entry point):
 *  - Status codes: QPR_OK (0) or a negative qpr_status; no C++ exception
 *    crosses the ABI; qpr_last_error() returns this thread's message for the
 *    last non-OK status.
 *  - Memory: the library never allocates or frees device memory at run time.
 *    The caller owns a problem arena (qpr_problem_bytes) and a workspace
 *    (qpr_workspace_bytes); both are device memory, 256-byte aligned.  The one
 *    exception is the static per-GPU array of qpr_rk4_step_noalloc, which the
 *    code object brings with it.  Solves read their control blocks back
 *    through small pinned host buffers (hipHostMalloc, freed before return).
 *  - Density matrices cross the ABI as planar FP64 device arrays of 2*n*n
 *    doubles: rho[a*n+b] = Re rho_ab, rho[n*n + a*n+b] = Im rho_ab (row-major,
 *    rho_ab = <a|rho|b>).  They must be Hermitian.
 *  - Streams: every call enqueues on `stream` (NULL = the null stream).
 *    qpr_rhs and qpr_rk4_step are asynchronous; qpr_build_google,
 *    qpr_steady_state, qpr_steady_state_many and qpr_batch_solve synchronise
 *    the streams they use.
 *  - Concurrency: calls that share a workspace must not overlap.
 */
#ifndef QPR_H
#define QPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* qpr_stream_t; /* the same type as hipStream_t */

typedef enum {
  QPR_OK = 0,
  QPR_E_ARG = -1,           /* invalid argument (message says which)          */
  QPR_E_HIP = -2,           /* a HIP runtime call failed                      */
  QPR_E_NOT_CONVERGED = -3, /* max_steps reached; rho holds the last state    */
  QPR_E_NONFINITE = -4,     /* NaN or Inf met in the state or right-hand side */
  QPR_E_UNSTABLE = -5,      /* dt outside the RK4 stability bound             */
  QPR_E_WORKSPACE = -6      /* arena or workspace too small                   */
} qpr_status;

/* Long-distance hopping ("teleport") matrix T of the Google matrix. */
typedef enum {
  QPR_TELEPORT_PAPER_F = 0, /* Eq. (S2): 1/(N-1) off the diagonal, 0 on it */
  QPR_TELEPORT_UNIFORM = 1  /* 1/N everywhere                               */
} qpr_teleport;

/* Hamiltonian of the coherent part. */
typedef enum {
  QPR_HDIAG_ZERO = 0, /* symmetrised adjacency max(A, A^T), zero diagonal     */
  QPR_HDIAG_PAPER = 1 /* Eq. (S6): -max(A_ij, A_ji), diagonal -outDeg(j)      */
} qpr_hdiag;

/* Arithmetic of the commutator product (the epilogue is always FP64). */
typedef enum {
  QPR_FP64 = 0,  /* FP64 matrix cores                                        */
  QPR_FP32 = 1,  /* FP32 matrix cores                                        */
  QPR_BF16X3 = 2 /* rho split in three bf16 slices, FP32 accumulation        */
} qpr_prec;

/*
 * A built problem.  Filled by qpr_build_google; the device pointers point into
 * the caller's arena, which must outlive every use of the struct.
 */
typedef struct {
  int32_t n;            /* nodes                                              */
  int32_t ld;           /* leading dimension of internal planes (n rounded up to 64) */
  int64_t n_edges_in;   /* edges passed in                                    */
  int64_t nnz_a;        /* distinct directed edges after dropping loops/duplicates */
  int64_t nnz_h;        /* nonzeros of the off-diagonal Hamiltonian           */
  int32_t n_self_loops; /* self-loops dropped                                 */
  int32_t n_dangling;   /* nodes without out-links                            */
  double alpha;         /* damping of the Google matrix                       */
  int32_t teleport;     /* qpr_teleport                                       */
  int32_t hdiag;        /* qpr_hdiag                                          */
  double h_lo, h_hi;    /* interval containing the spectrum of H: Gershgorin's,
                           narrowed to [-b, b] by a Collatz-Wielandt bound b on
                           its spectral radius (the RK4 stability check uses it) */
  double h_norm;        /* spectral radius of H, power-iteration estimate     */
  int32_t pagerank_iters; /* power iterations used for `pagerank`             */
  int32_t reserved;
  /* device arrays inside the arena */
  double* h_off;        /* ld*ld, off-diagonal H (0 or +-1), zero padded      */
  float* h_off_f32;     /* ld*ld, the same values in FP32                     */
  uint16_t* h_off_bf16; /* ld*ld, the same values in bf16                     */
  double* h_diag;       /* n, diagonal of H                                   */
  double* d;            /* n, column sums of G                                */
  double* inv_outdeg;   /* n, 1/outDeg(j), 0 for a dangling node              */
  int32_t* dangling;    /* n, 1 if node j has no out-links                    */
  int32_t* outdeg;      /* n                                                  */
  int32_t* indeg;       /* n                                                  */
  int32_t* in_ptr;      /* n+1, CSR of in-links: row a lists j with j -> a     */
  int32_t* in_idx;      /* nnz_a, ascending within a row                      */
  int32_t* out_ptr;     /* n+1, CSR of out-links: row j lists a with j -> a    */
  int32_t* out_idx;     /* nnz_a                                              */
  double* pagerank;     /* n, stationary vector of G (power iteration)        */
  int32_t* h_ptr;       /* n+1, CSR pattern of H_off (all values equal: +1 or -1) */
  int32_t* h_idx;       /* nnz_h, ascending within a row                      */
  void* arena;
  size_t arena_bytes;
} qpr_problem;

/* Per-solve statistics (host struct). */
typedef struct {
  int64_t steps;          /* RK4 steps taken (the state returned is y_steps)  */
  int64_t rhs_evals;      /* right-hand-side evaluations, all precisions      */
  int64_t rhs_evals_fp64; /* of which with the FP64 product                   */
  int64_t folds;          /* defect-correction folds (mixed precision)        */
  double t;               /* integrated time                                  */
  double residual;        /* ||L(rho)||_F of the returned state, FP64         */
  double trace_err;       /* |tr rho - 1| of the returned state               */
  double herm_err;        /* max |rho - rho^dag| of the returned state        */
  double min_diag;        /* min_a Re rho_aa                                  */
  double seconds;         /* host wall time of the call                       */
  int32_t converged;      /* 1 if residual < tol                              */
  int32_t status;         /* qpr_status of the call                           */
  int64_t rejected;       /* adaptive integration: rejected step attempts     */
  double last_step;       /* adaptive integration: step size at the end       */
} qpr_stats;

/* Solver options; pass NULL for the defaults in brackets. */
typedef struct {
  int32_t chunk;      /* RK4 steps per host check of the device flag [64]     */
  int32_t use_graph;  /* replay each chunk as a captured HIP graph [1]        */
  int32_t fold_every; /* mixed precision: steps between FP64 folds [=chunk]   */
  int32_t renorm;     /* mixed precision: divide by the trace at folds [1]    */
  int32_t gemm_cfg;   /* product tile configuration (qpr_product_configs), -1 =
                         tuned default [-1]; an index past the table takes the
                         default, a tile that does not divide the padded size
                         configuration 0 (64 x 64, divides every padded size);
                         qpr_batch_solve's persistent form has its own three   */
  int32_t product;    /* qpr_product [QPR_PRODUCT_AUTO]                       */
  int32_t integrator; /* qpr_integrator [QPR_RK4]                             */
  int32_t sparse_variant; /* sparse product kernel variant + 1, 0 = default [0];
                             variants as listed under qpr_time_kernels;
                             single-system calls only                    */
  int32_t batch_mode;    /* qpr_batch_solve: qpr_batch_mode [QPR_BATCH_AUTO]  */
  int32_t batch_workers; /* qpr_batch_solve, concurrent form: worker threads and
                            streams, 0 = min(nsys, 8), at most 64 [0]        */
  double step_tol;    /* RKF45: local error tolerance per unit step [1e-4]    */
  double dt_max;      /* RKF45: step cap; 0 = from the spectral radius of H [0] */
  int32_t delta_state; /* mixed precision (QPR_FP32): storage of the defect delta,
                          its RK4 stage states, accumulator and the copy of r_a
                          the steps add: 1 FP64 (the stage writes an FP32 copy for
                          the product), 2 FP32 (every state plane of the steps
                          single precision, arithmetic FP64; needs the sparse
                          product), 0 = FP32 with QPR_PRODUCT_AUTO where the
                          product is sparse, else FP64 [0].  qpr_steady_state,
                          qpr_steady_state_many and both batch forms (the
                          persistent one decides on the largest system)     */
  int32_t reserved;
} qpr_opts;

/* Time integrator of qpr_steady_state. */
typedef enum {
  QPR_RK4 = 0,   /* classical RK4, fixed step dt (Supplementary Note 2)       */
  QPR_RKF45 = 1  /* Fehlberg 4(5) with the step control of Eq. (S13): dt is the
                    first step; the two 4101 denominators read as 4104; FP64 */
} qpr_integrator;

/* How the commutator product X = H_off rho is formed.  The sparse product
 * serves QPR_FP64 (FP64 operand) and QPR_FP32 (gathers of the FP32 copy of
 * the state, sums in FP64, X rounded to FP32); QPR_BF16X3 is always dense. */
typedef enum {
  QPR_PRODUCT_AUTO = 0,   /* sparse when H_off is below 5 % dense, else dense; the sparse
                             choice is FUSED for the FP32 steps of the mixed solve, and for
                             FP64 stages from a padded size of 4096 on, in qpr_batch_solve,
                             and in qpr_steady_state_many while two or more systems run */
  QPR_PRODUCT_DENSE = 1,  /* dense MFMA product, then the epilogue (two launches per stage) */
  QPR_PRODUCT_SPARSE = 2, /* CSR gathers: X row a = sum of the rows of rho listed for a in H_off */
  QPR_PRODUCT_FUSED = 3,  /* the same gathers inside the epilogue: each tile pair gathers the two
                             32 x 32 blocks of X it needs into LDS, so X never goes to HBM and a
                             stage is one launch; bitwise the SPARSE stage.  The FP32 steps
                             of the mixed solve gather the FP32 copy of the state the same way
                             (X rounded once to FP32, as the separate FP32 product) */
  QPR_PRODUCT_BLOCKSPARSE = 4 /* the MFMA product with tile skipping: each 32-row block of H_off
                             multiplies only the 16-wide k-slabs in which it has a nonzero (slab
                             lists built from the CSR pattern at the start of the call); equal to
                             the dense product.  QPR_FP64 and QPR_FP32 (FP32 operands); not the
                             persistent batch form */
} qpr_product;

/* How qpr_batch_solve runs its systems. */
typedef enum {
  QPR_BATCH_AUTO = 0,       /* the persistent form for QPR_FP32 batches of 8 or more
                               systems with QPR_PRODUCT_AUTO and the defect not forced
                               to FP64 (1.2-1.35x faster there), else the concurrent
                               form (faster on every FP64 batch measured)              */
  QPR_BATCH_PERSISTENT = 1, /* shared persistent launches over (system, tile) work lists,
                               chunks replayed as one captured graph for all systems   */
  QPR_BATCH_CONCURRENT = 2  /* single-system solves on a pool of worker streams, as
                               qpr_steady_state_many                                   */
} qpr_batch_mode;

/* ------------------------------------------------------------------ build */

/* Bytes of the problem arena for n nodes and n_edges input edges. */
size_t qpr_problem_bytes(int32_t n, int64_t n_edges);

/*
 * Build the Google matrix G = alpha S + (1-alpha) T (Eq. (S4) read as the
 * column-stochastic Google matrix; S is the out-degree-normalised adjacency of
 * Supplementary Note 1, a dangling column takes the teleport column), the
 * Hamiltonian of Eq. (S6) per `hdiag`, the column sums d of G and the PageRank
 * vector of G by power iteration.
 *   n        number of nodes, n >= 2
 *   src,dst  HOST arrays of n_edges int32: edge src[e] -> dst[e], meaning
 *            A[dst][src] = 1 (Supplementary Note 1).  0 <= src,dst < n.
 *            Duplicates collapse; self-loops are dropped and counted.
 *   alpha    in [0, 1]
 *   arena    device memory of at least qpr_problem_bytes(n, n_edges)
 *   out      host struct filled on QPR_OK
 * Errors: QPR_E_ARG (n < 2, bad alpha/teleport/hdiag, edge out of range, NULL
 * pointer), QPR_E_WORKSPACE (arena too small), QPR_E_HIP.  Synchronises.
 */
qpr_status qpr_build_google(int32_t n, int64_t n_edges, const int32_t* src,
                            const int32_t* dst, double alpha, int32_t teleport,
                            int32_t hdiag, void* arena, size_t arena_bytes,
                            qpr_problem* out, qpr_stream_t stream);

/* Bytes of workspace a call on an n-node problem needs at precision prec with
 * integrator `integrator` (qpr_integrator; QPR_RKF45 adds the Fehlberg stage
 * planes and is FP64 only; qpr_rhs, qpr_rk4_step, qpr_time_kernels and
 * qpr_autotune need the QPR_RK4 size).  0 for an invalid request. */
size_t qpr_workspace_bytes(int32_t n, int32_t prec, int32_t integrator);

/* ------------------------------------------------------------------ solve */

/*
 * out = L(rho), the right-hand side of Eq. (1) (reading above), with the
 * commutator product at precision `prec` and everything else in FP64.
 *   rho, out  device, 2*n*n planar FP64 (may not alias)
 * Errors: QPR_E_ARG (omega outside [0,1], NULL), QPR_E_WORKSPACE, QPR_E_HIP.
 * Asynchronous.
 */
qpr_status qpr_rhs(const qpr_problem* P, double omega, const double* rho,
                   double* out, int32_t prec, const qpr_opts* opts, void* ws,
                   size_t ws_bytes, qpr_stream_t stream);

/*
 * nsteps classical RK4 steps of size dt (Supplementary Note 2) applied to rho
 * in place.  If diag_out (device, 4 doubles) is not NULL it receives
 * [ ||L(y)||_F^2 at the start of the last step, tr y_final, max|y - y^dag|,
 * nonfinite flag ] of the final state.
 * Errors: QPR_E_ARG, QPR_E_UNSTABLE, QPR_E_WORKSPACE, QPR_E_HIP.
 * Asynchronous.
 */
qpr_status qpr_rk4_step(const qpr_problem* P, double omega, double dt,
                        int32_t nsteps, double* rho, int32_t prec,
                        double* diag_out, const qpr_opts* opts, void* ws,
                        size_t ws_bytes, qpr_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * qpr_rk4_step with its workspace in a static device array the library
 * holds on every GPU it runs on (73 MiB each, for the life of the
 * process) instead of a caller buffer.  Same arguments and results as
 * qpr_rk4_step without ws/ws_bytes; prec must be QPR_FP64 and n <= 1024.
 * Calls no allocating routine.  All calls on one GPU share that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race; calls
 * on one stream run in order.  Nothing a previous call left in the array is
 * read.
 * Errors: those of qpr_rk4_step; QPR_E_ARG for n > 1024 or prec != QPR_FP64.
 * Asynchronous.
 */
qpr_status qpr_rk4_step_noalloc(const qpr_problem* P, double omega, double dt,
                                int32_t nsteps, double* rho, int32_t prec,
                                double* diag_out, const qpr_opts* opts,
                                qpr_stream_t stream);

/*
 * Integrate from rho (in: rho0) until the first step n with
 * ||L(y_n)||_F < tol, FP64-judged, and return y_n in rho.  With prec != FP64
 * the solve is a defect correction: an FP64 anchor rho_a with FP64 residual
 * r_a = L(rho_a), and d delta/dt = r_a + L_prec(delta) integrated with the
 * low-precision product, folded into the anchor (and trace-renormalised) every
 * opts->fold_every steps; convergence is judged on the FP64 residual.
 *   rank   device int32[n] or NULL: nodes by descending Re rho_aa, ties by
 *          ascending index (computed in FP64)
 *   stats  host, may be NULL
 *   opts   may be NULL
 * Errors: QPR_E_ARG, QPR_E_UNSTABLE, QPR_E_WORKSPACE, QPR_E_HIP,
 * QPR_E_NONFINITE, QPR_E_NOT_CONVERGED (rho then holds the last state so the
 * call can be resumed).  Synchronises once per chunk.
 */
qpr_status qpr_steady_state(const qpr_problem* P, double omega, double dt,
                            double tol, int64_t max_steps, int32_t prec,
                            double* rho, int32_t* rank, qpr_stats* stats,
                            const qpr_opts* opts, void* ws, size_t ws_bytes,
                            qpr_stream_t stream);

/*
 * `count` independent qpr_steady_state solves run concurrently by a pool of
 * `nworkers` host threads (on the caller's current device): worker w solves
 * on streams[w] with workspace ws[w], taking the next unsolved system (index
 * order) whenever it is free, so min(nworkers, systems left) run at once.
 * Small systems leave most of the GPU idle between dependent launches;
 * kernels of the other systems fill it.  Every system computes exactly what
 * qpr_steady_state computes on it (bitwise the same state, rank and step
 * count).  With QPR_PRODUCT_AUTO, FP64 stages that a lone solve would give the
 * sparse product + epilogue take the fused epilogue (QPR_PRODUCT_FUSED, the
 * same sums in the same order) while two or more systems run, the faster
 * form when other systems' kernels run beside it; a system left running
 * alone goes back to the two kernels.
 *   probs, omegas, rhos, ranks  HOST arrays [count]; rhos[k] device planar
 *           2*n_k*n_k FP64 (in: rho0, out: steady state); ranks may be NULL
 *           or hold NULL entries
 *   stats   HOST qpr_stats[count] or NULL
 *   nworkers  1..64 (more than count is allowed; count are used)
 *   ws, ws_bytes, streams  HOST arrays [nworkers]: distinct streams, and
 *           non-overlapping 256-byte-aligned workspaces of at least
 *           qpr_workspace_bytes(largest n, prec, opts->integrator) bytes each
 * Returns QPR_OK when every system returns QPR_OK, else the status of the
 * lowest-numbered failing system, whose message qpr_last_error() gives
 * (prefixed "system k: "); stats[k].status holds each system's own status.
 * Errors: those of qpr_steady_state, QPR_E_ARG (count < 1, nworkers out of
 * range, NULL arrays, a repeated stream), QPR_E_WORKSPACE (a workspace too
 * small for the largest system).  Returns when every system has finished.
 * With the environment variable QPR_PROGRESS set to a number of seconds, the
 * count of finished systems is printed to stderr at most that often, and
 * when the last one finishes if the run lasted that long; unset, nothing is
 * printed.
 */
qpr_status qpr_steady_state_many(int32_t count, const qpr_problem* const* probs,
                                 const double* omegas, double dt, double tol,
                                 int64_t max_steps, int32_t prec,
                                 double* const* rhos, int32_t* const* ranks,
                                 qpr_stats* stats, const qpr_opts* opts,
                                 int32_t nworkers, void* const* ws,
                                 const size_t* ws_bytes, const qpr_stream_t* streams);

/* Bytes of workspace qpr_batch_solve needs for systems of sizes n[0..nsys)
 * with these options (NULL = defaults): the concurrent form takes one
 * qpr_workspace_bytes(largest n, prec, integrator) per worker; the persistent form one
 * workspace per system (opts->integrator = QPR_RKF45 adding each system's
 * Fehlberg stage planes) plus its work lists.  0 for an invalid request. */
size_t qpr_batch_workspace_bytes(int32_t nsys, const int32_t* n, int32_t prec,
                                 const qpr_opts* opts);

/*
 * Solve nsys independent systems (problem probs[k] at omega omegas[k]) to the
 * steady state of Eq. (1) with RK4 (Supplementary Note 2) or, with
 * opts->integrator = QPR_RKF45 (FP64 only), the adaptive Fehlberg 4(5) of
 * qpr_steady_state with a step size and step control per system (dt = first
 * step, cap from the system's spectral bound unless opts->dt_max > 0).
 * prec QPR_FP64 or QPR_FP32 (the FP32 product with the FP64 fold-and-judge
 * defect correction of qpr_steady_state).  Two forms (opts->batch_mode;
 * QPR_BATCH_AUTO takes the persistent one for QPR_FP32 batches of 8 or more
 * systems with QPR_PRODUCT_AUTO and delta_state not 1, the concurrent one
 * otherwise):
 *  - concurrent (QPR_BATCH_CONCURRENT): single-system solves
 *    on a pool of opts->batch_workers worker threads, each with a stream of
 *    its own (created here, ordered after `stream`) and a workspace of its
 *    own carved from ws, as qpr_steady_state_many; each system bitwise its
 *    lone qpr_steady_state solve; opts->chunk steps per host check [64];
 *  - persistent (QPR_BATCH_PERSISTENT): shared launches in which every stage
 *    kernel covers all running systems through a device-side (system, tile)
 *    work list; chunks of opts->chunk steps [32] (RKF45: attempts) are
 *    replayed as one captured HIP graph, and between replays the lists are
 *    shrunk to the systems still running; the product follows opts->product,
 *    decided on the largest system's density for the whole batch (with AUTO the sparse
 *    stages, FP64 and FP32, run as fused epilogues); a dense product runs one
 *    of three tile configurations per precision (64 x 64 tiles with 16- or
 *    32-deep k-slabs, 32 x 32 tiles): opts->gemm_cfg 0..2 picks it (larger is
 *    QPR_E_ARG), a negative value times each on this batch's own work list
 *    and takes the fastest.  FP64: bitwise the lone solves; FP32: the defect
 *    held as opts->delta_state says, as in the lone solve (its fold of the
 *    defect into the anchor is one kernel here, so the step counts can
 *    differ slightly from the lone solve's).
 *   probs, omegas, rhos, ranks  HOST arrays of nsys entries; rhos[k] are
 *           device planar 2*n_k*n_k FP64 (in: rho0, out: steady state); ranks
 *           may be NULL or hold device int32[n_k] / NULL entries
 *   stats   HOST qpr_stats[nsys] or NULL (per-system status in stats[k].status)
 *   tuned_cfg  HOST int32 or NULL: the persistent form's dense tile
 *           configuration, as the index opts->gemm_cfg takes (-1 without a
 *           dense product, and always -1 in the concurrent form)
 *   tune_cache  HOST path or NULL: a cache written by qpr_autotune, loaded
 *           (qpr_load_tuning) before the solve, so its dense tiles, sparse
 *           variants and stage forms are the ones the batch uses; NULL keeps
 *           the process's current tuning
 * Errors: QPR_E_ARG, QPR_E_UNSTABLE, QPR_E_WORKSPACE, QPR_E_HIP, and after a
 * full run QPR_E_NONFINITE / QPR_E_NOT_CONVERGED if any system failed.
 * Synchronises once per chunk.  QPR_PROGRESS=<seconds> in the environment
 * prints the count of finished (concurrent) or stopped (persistent) systems
 * to stderr at most that often, as qpr_steady_state_many does.
 */
qpr_status qpr_batch_solve(int32_t nsys, const qpr_problem* const* probs,
                           const double* omegas, double dt, double tol,
                           int64_t max_steps, int32_t prec, double* const* rhos,
                           int32_t* const* ranks, qpr_stats* stats,
                           const qpr_opts* opts, int32_t* tuned_cfg,
                           const char* tune_cache, void* ws, size_t ws_bytes,
                           qpr_stream_t stream);

/*
 * Rank nodes by descending p (device, n doubles), ties by ascending index,
 * into order (device int32[n]).  Asynchronous.
 */
qpr_status qpr_rank(int32_t n, const double* p, int32_t* order,
                    qpr_stream_t stream);

/* ------------------------------------------------------- learned warm start */
/*
 * A small message-passing network predicts diag(rho_ss) so the integrator
 * can start from rho0 = diag(p_hat) (the FP64 solve still finishes and judges;
 * the paper has no learned part).  Per node i:
 *   x_i  = [log(1+in_i), log(1+out_i), N * PageRank_i, omega]
 *   h'_i = ReLU(Ws h_i + Win mean_{j->i} h_j + Wout mean_{i->j} h_j + b)  (3 layers, width 64)
 *   s_i  = w . h_i + c,  p_hat = softmax(s) within each graph
 *   loss = mean over graphs of KL(p || p_hat)
 * Parameters are one FP32 array of qpr_mpnn_param_count() values:
 * for l = 0,1,2: Ws_l, Win_l, Wout_l (each 64 x F_l row-major, F_0 = 4,
 * F_1 = F_2 = 64), b_l (64); then w (64) and c (1).
 * A batch is block-diagonal: graphs are concatenated and node ids are global.
 */
typedef struct {
  int32_t n_nodes;         /* total nodes                                    */
  int32_t n_graphs;        /* graphs                                         */
  const float* x;          /* n_nodes x 4 features (qpr_mpnn_features)       */
  const int32_t* in_ptr;   /* n_nodes+1; row i lists j with j -> i           */
  const int32_t* in_idx;
  const int32_t* out_ptr;  /* n_nodes+1; row i lists j with i -> j           */
  const int32_t* out_idx;
  const float* inv_in;     /* 1/in-degree (0 if none)                        */
  const float* inv_out;    /* 1/out-degree (0 if none)                       */
  const int32_t* graph_ptr;/* n_graphs+1 node offsets                         */
} qpr_mpnn_batch;          /* every pointer is device memory                  */

int32_t qpr_mpnn_param_count(void);
/* workspace (device) for one forward + backward over a batch of this size */
size_t qpr_mpnn_workspace_bytes(int32_t n_nodes, int32_t n_graphs);
/* features x (n x 4), inv_in, inv_out (n) of one built problem, on device */
qpr_status qpr_mpnn_features(const qpr_problem* P, double omega, float* x,
                             float* inv_in, float* inv_out, qpr_stream_t stream);
/* forward pass; p_hat (device, n_nodes) may be NULL; keeps activations in ws */
qpr_status qpr_mpnn_forward(const qpr_mpnn_batch* batch, const float* params,
                            float* p_hat, void* ws, size_t ws_bytes,
                            qpr_stream_t stream);
/* backward pass after qpr_mpnn_forward on the same ws: grads (device,
   param_count) = d loss / d params; loss (device, 1 float) may be NULL.
   Deterministic: fixed-order reductions, no floating-point atomics. */
qpr_status qpr_mpnn_backward(const qpr_mpnn_batch* batch, const float* params,
                             const float* p_true, float* grads, float* loss,
                             void* ws, size_t ws_bytes, qpr_stream_t stream);
/* one Adam step (Kingma & Ba), step counted from 1, on device arrays */
qpr_status qpr_mpnn_adam(float* params, const float* grads, float* m, float* v,
                         int32_t count, int32_t step, float lr, float b1,
                         float b2, float eps, qpr_stream_t stream);

/* ---------------------------------------------------------- measurement */

/*
 * Time the two kernels of the RK4 stages on `stream` with HIP events: `reps`
 * back-to-back launches of the commutator product X = H_off [Re rho | Im rho]
 * (the real products of the coherent term of Eq. (1)) at precision `prec`
 * with tile configuration `cfg` (-1 = default), then the fused epilogues of
 * `reps` classical RK4 steps (stages 1-4 in turn, stage 1 with its residual,
 * trace and finiteness reductions; X held fixed; each reads Y_s, y_n and the
 * accumulator, writes the accumulator and Y_{s+1}, plus X
 * for the dense product).  cfg = -2 with QPR_FP64 or QPR_FP32 times the
 * sparse product (CSR gathers of rho through the pattern of H_off) in place
 * of the dense one;
 * cfg = -3 - v times sparse-product variant v: 0 cm_w32_r1, 1 cm_w64_r1,
 * 2 cm_w128_r1, 3 cm_w64_r2 (column-chunk major, XCD-aware: W columns of
 * both planes per wave, R rows per wave), 4 row128 (one workgroup per row and
 * 128-column chunk).  The default is row128 below N = 1536 and cm_w128_r1 above where
 * the padded size is a multiple of 128.  All variants give bitwise the same
 * product.  With QPR_FP64 or QPR_FP32, v = qpr_sparse_variants() times the
 * fused epilogue of QPR_PRODUCT_FUSED (no product launch: ms_out[0] = 0);
 * v = qpr_sparse_variants() + 1 times the block-sparse product of
 * QPR_PRODUCT_BLOCKSPARSE in place of the dense one; with QPR_FP32,
 * v = qpr_sparse_variants() + 2 times the fused stages of the defect held in
 * FP32 (opts delta_state; no product launch).
 *   rho     device, 2*n*n planar FP64 operand (unchanged)
 *   ms_out  HOST double[2]: mean milliseconds per product launch and per
 *           epilogue launch (the mean over the four stages)
 * Errors: QPR_E_ARG, QPR_E_WORKSPACE, QPR_E_HIP.  Synchronises.
 */
qpr_status qpr_time_kernels(const qpr_problem* P, double omega, int32_t prec,
                            int32_t cfg, int32_t reps, const double* rho,
                            double* ms_out, void* ws, size_t ws_bytes,
                            qpr_stream_t stream);

/*
 * Autotuner: time every dense-product tile configuration at precision prec on
 * P's padded size (`reps` launches each, HIP events on `stream`), make the
 * fastest the default for that (precision, size) in this process and, if
 * cache_path is not NULL, append "prec ld cfg microseconds name" to it.
 * With QPR_FP64 it also times every sparse-product variant (the fastest
 * becomes the default for this size: line "10 ld variant us name") and the
 * two forms of a sparse RK4 stage, product + epilogue against the fused
 * epilogue (what QPR_PRODUCT_AUTO runs for a lone FP64 solve of this size:
 * line "11 ld 0|1 us-per-stage name").
 *   best_cfg  host int32 or NULL;  us_out  host double[qpr_product_configs(prec)]
 *             or NULL (-1 for configurations whose tile does not divide ld)
 * Errors: QPR_E_ARG, QPR_E_WORKSPACE, QPR_E_HIP.  Synchronises.
 */
qpr_status qpr_autotune(const qpr_problem* P, int32_t prec, int32_t reps,
                        const char* cache_path, int32_t* best_cfg, double* us_out,
                        void* ws, size_t ws_bytes, qpr_stream_t stream);
/* Load a cache written by qpr_autotune (later lines win). */
qpr_status qpr_load_tuning(const char* cache_path);

/* Number of product tile configurations at precision prec (0 for an unknown
 * precision), and their names ("?" for an unknown precision or index). */
int32_t qpr_product_configs(int32_t prec);
const char* qpr_product_config_name(int32_t prec, int32_t cfg);

/* Number of sparse-product kernel variants (qpr_opts.sparse_variant - 1,
 * qpr_time_kernels cfg -3 - v), and their names; NULL for an invalid v. */
int32_t qpr_sparse_variants(void);
const char* qpr_sparse_variant_name(int32_t v);

/*
 * Hub classes of the results section: counts[0] = #{i : p_i > c/N} (main
 * hubs), counts[1] = #{i : 1/N < p_i <= c/N} (secondary hubs); the paper
 * uses c = 10.  p device n doubles, counts device int32[2].  Asynchronous.
 */
qpr_status qpr_hub_counts(int32_t n, const double* p, double c, int32_t* counts,
                          qpr_stream_t stream);

/* Message for this thread's last non-OK status ("" if none). */
const char* qpr_last_error(void);

/* Library version string. */
const char* qpr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QPR_H */
