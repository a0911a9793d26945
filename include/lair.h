/*
 * lair.h -- C ABI of liblair, an MI355X (gfx950) implementation of the
 * data-parallel hot path of lAIR: nonsymmetric algebraic multigrid with
 * local approximate ideal restriction and F-relaxation (Manteuffel, Ruge,
 * Southworth, arXiv:1708.06065).
 *
 * The library builds a multigrid hierarchy on the GPU from a square sparse
 * matrix A (CSR) and a CF splitting, and runs V-cycles with F-F-C Jacobi
 * relaxation:
 *   setup  (per level)  strength of connection (Sec. 4), restriction
 *                        neighbourhoods (Sec. 3.1 / Sec. 4), one dense local
 *                        solve per C-point (Eq. (system)) giving R = [Z I]
 *                        (Eq. (PR)), interpolation P, Galerkin K = R A P
 *                        (Sec. 2.1);
 *   cycle               coarse-grid correction x += P K^{-1} R (b - A x)
 *                        (Sec. 2.1) followed by Jacobi on F, F, then C points
 *                        (Sec. 4, relaxation paragraph).
 *
 * Conventions for every entry point:
 *  - Matrices are CSR with int32 row pointers and column indices and double
 *    values; each row's columns are strictly increasing and the diagonal is
 *    stored.  Vectors are double.  Several right-hand sides are interleaved:
 *    element (i, k) of an n x nrhs block is at [i * nrhs + k].
 *  - Pointers named "device" are HIP device pointers on the current device.
 *    The caller owns every buffer it passes; the library never keeps a
 *    caller pointer beyond the call (lair_setup copies A).
 *  - `stream` is a hipStream_t (NULL = the null stream).  All device work of
 *    a call is ordered on it; calls that report results to the host
 *    synchronise it before returning.
 *  - Errors are returned as lair_status codes; no exception or abort crosses
 *    the ABI.  Arguments are validated before any device work.  A message for
 *    the last failure on the calling thread is available from
 *    lair_last_error().
 *  - One hierarchy may be used by one stream at a time; distinct hierarchies
 *    are independent.
 */
#ifndef LAIR_H
#define LAIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lair_status;

#define LAIR_OK             0
#define LAIR_EINVAL        -1   /* invalid argument or malformed input      */
#define LAIR_ENOMEM        -2   /* device or host allocation failed         */
#define LAIR_EDEVICE       -3   /* HIP runtime error / no device            */
#define LAIR_ESINGULAR     -4   /* coarsest-grid matrix is singular         */
#define LAIR_ENOCONV       -5   /* tolerance not reached within maxit       */
#define LAIR_EUNSUPPORTED  -6   /* a size limit of this build was exceeded  */

/* strength-of-connection kinds (Sec. 4) */
#define LAIR_SOC_ABS 0   /* |a_ij| >= theta max_{k!=i} |a_ik|                */
#define LAIR_SOC_NEG 1   /* -a_ij  >= theta max_{k!=i} |a_ik|  (paper's form) */

/* neighbourhood distance for R (Sec. 3.1): 1, 2, or every F-point */
#define LAIR_DIST_ALL_F 0

/* interpolation */
#define LAIR_P_ONE_POINT 0  /* value of the strongest C-neighbour (Sec. 4) */
#define LAIR_P_DIRECT    1  /* classical direct interpolation              */

/* precision of the setup's local solves and of the cycle */
#define LAIR_FP64        0  /* everything in double                        */
#define LAIR_MIXED       1  /* float local LU + one double refinement step
                               per row of Z; float cycle under a double outer
                               iteration (residual, update, norms in double) */
#define LAIR_MIXED_LOCAL 2  /* float local LU + one double refinement step
                               per row of Z; the cycle in double           */

/* A square CSR matrix handed to lair_setup. */
typedef struct lair_csr {
    int64_t n;               /* rows = columns, 1 <= n < 2^31               */
    int64_t nnz;             /* stored entries, nnz < 2^31                  */
    const int32_t *rowptr;   /* n + 1 offsets, rowptr[0] = 0                */
    const int32_t *col;      /* nnz column indices, sorted, unique per row  */
    const double *val;       /* nnz values, finite                          */
    int32_t on_device;       /* 1: the three arrays are device pointers     */
} lair_csr;

/* Strength of connection and neighbourhood (Sec. 3.1, Sec. 4). */
typedef struct lair_strength {
    double theta;            /* threshold for neighbourhoods and P  (0.25)  */
    double theta_c;          /* threshold for the library's own CF split    */
    int32_t kind;            /* LAIR_SOC_ABS or LAIR_SOC_NEG                */
    int32_t distance;        /* 1, 2 or LAIR_DIST_ALL_F                     */
} lair_strength;

/* Optional per-level CF splittings.  Level l uses cf[offs[l] .. offs[l+1])
 * with 1 = C-point, 0 = F-point; its length must equal that level's size.
 * Levels beyond nlevels use the library's own splitting.  offs is host
 * memory; cf is host memory, or device memory when on_device is 1 (then
 * checked and counted on the device, with no host pass over it). */
typedef struct lair_cf_levels {
    int32_t nlevels;
    const int64_t *offs;     /* nlevels + 1 entries (host)                   */
    const int8_t *cf;
    int32_t on_device;       /* 1: cf is a device pointer                    */
} lair_cf_levels;

typedef struct lair_options {
    int32_t interp;          /* LAIR_P_ONE_POINT or LAIR_P_DIRECT           */
    int32_t precision;       /* LAIR_FP64 or LAIR_MIXED                     */
    double omega;            /* Jacobi weight (1.0)                         */
    int32_t max_levels;      /* at most this many levels (25)               */
    int32_t max_coarse;      /* stop coarsening at n <= max_coarse (128)    */
    double stall;            /* stop when n_c > stall * n (0.9)             */
    int32_t block_size;      /* 0, or k: solve D_B^{-1} A x = D_B^{-1} b with
                                D_B the k x k diagonal blocks (Sec. 4.2.1);
                                the diagonal blocks of D_B^{-1} A are stored
                                as the exact identity                      */
    int32_t flags;           /* 0, or LAIR_FLAG_* bits below                */
    double lump_tol;         /* 0 (off), or theta_D in (0, 1]: every coarse
                                operator drops the off-diagonal entries of a
                                row below theta_D times the row's largest
                                magnitude (diagonal included) and adds them
                                to the diagonal, keeping row sums (Sec. 3.3
                                and its filtering table; the paper's results
                                use 0.001)                                 */
} lair_options;

/* Solves capture one iteration (cycle, residual, norms) in a HIP graph the
 * first time a (b, x, nrhs) combination is seen, on a private stream of
 * default priority, and replay it on the caller's stream afterwards; the
 * results are bitwise those of eager launches.  This flag launches every
 * kernel eagerly instead.  Iterations are also eager while the profiler
 * times a cycle category. */
#define LAIR_FLAG_NO_GRAPH 1
/* A single system's cycle runs, on its large levels (n >= 65536, a prefix
 * of the hierarchy), on
 * copies of A_l, R_l and P_l renumbered with each level's F-points first and
 * its C-points after them (both ascending), so that the F and C sweeps of
 * FF C-relaxation read and write contiguous blocks; every row keeps its
 * entries in stored order, so the cycle's sums are those of the natural
 * ordering and the results are bitwise the same.  b and x stay in the
 * caller's (natural) ordering.  NATURAL_ORDER runs every level on the
 * natural matrices (batches always do); SPLIT_ALL renumbers every level but
 * the coarsest whatever its size. */
#define LAIR_FLAG_NATURAL_ORDER 2
#define LAIR_FLAG_SPLIT_ALL 4
/* With block_size = k: build the hierarchy by k x k blocks (the nodal
 * treatment of Sec. 4.2, with R from the block form of Eq. (system) in
 * Sec. 3.1) instead of scaling by the block diagonal.  The k rows of node i
 * are rows i k .. i k + k - 1; they must store the same columns in whole
 * dense blocks (explicit zeros included), else setup fails with
 * LAIR_EINVAL.  Block (i, j) is strong when
 * ||A_ij||_F^2 >= theta^2 max_{l != i} ||A_il||_F^2 (the squares summed row by
 * row, without fused multiply-adds); the first pass splits the graph of
 * blocks, every row of a node taking the node's type (caller splittings must
 * do the same); N_i holds every row of the strong F-neighbour nodes (and of
 * theirs at distance 2, F-F-C paths on the graph of blocks), so the
 * k rows of C-node i solve the same system A(N,N)^T with k right-hand sides;
 * an F-node takes the identity block from its strong C-neighbour with the
 * largest block norm (one-point interpolation by block, ties to the first);
 * the sweeps are block Jacobi, x_X + omega D_X^{-1} (b - A x)_X.  Needs
 * interp = LAIR_P_ONE_POINT, distance 1 or 2 and no lumping; single systems only;
 * no transposed cycle or solve and no new diagonal (LAIR_EUNSUPPORTED).
 * Natural ordering on every level. */
#define LAIR_FLAG_NODAL 8
/* Levels without a caller splitting are split on the device by a parallel
 * splitting of the PMIS type (De Sterck, Yang and Heys, 2006) instead of the
 * sequential Ruge-Stueben first pass of Sec. 4 on the host.  Weight of point
 * i: the number of points that strongly depend on it, then MurmurHash3's
 * 32-bit finalizer of i, then i.  Points on which nothing strongly depends
 * are F; each round, every undecided point that beats every undecided point
 * it is strongly connected to (either direction) becomes C, then every
 * undecided point that strongly depends on a C-point becomes F.  The result
 * does not depend on thread order.  It is a different coarsening from the
 * paper's, usually coarser.  Not with LAIR_FLAG_NODAL (LAIR_EUNSUPPORTED). */
#define LAIR_FLAG_PMIS 16

#define LAIR_HIST_MAX 256

typedef struct lair_info {
    int32_t iters;           /* V-cycles done                               */
    int32_t nlevels;
    double relres;           /* max over right-hand sides of
                                ||b - A x||_2 / ||b||_2 at return          */
    double rho;              /* geometric-mean residual reduction / cycle   */
    double cycle_complexity; /* work units per cycle (1 WU = SpMV with A_0) */
    double op_complexity;    /* sum_l nnz(A_l) / nnz(A_0)                   */
    int64_t n_singular_local;/* local systems solved by least squares       */
    double setup_ms;         /* wall time of lair_setup                     */
    double solve_ms;         /* wall time of the last solve                 */
    double split_ms;         /* host wall time lair_setup spent in the
                                library's own sequential CF splittings (the
                                classical first pass, with the copies of
                                the pattern it needs); 0 when every level's
                                splitting was given or split on the device */
    double wpd;              /* work units per digit of accuracy,
                                -cycle_complexity / log10(rho) (Sec. 4, the
                                solver-efficiency measure); 0 when rho is 0
                                or rho >= 1                                */
    double setup_phase_ms[8];/* host wall time of lair_setup by phase (the
                                waits for the device included): [0] copy,
                                checks and block scaling of A, [1] strength
                                and splitting, [2] neighbourhoods,
                                interpolation and local solves, [3]
                                Galerkin products and lumping, [4] coarsest
                                factors, [5] the cycle's operators and
                                statistics, [6..7] 0                       */
    int32_t hist_len;        /* entries of relres_hist: min(iters + 1,
                                LAIR_HIST_MAX); 0 for lair_solve_fgmres    */
    double relres_hist[LAIR_HIST_MAX]; /* largest relative residual over the
                                right-hand sides (over the systems of a
                                batch) before the first cycle, then after
                                each cycle                                 */
} lair_info;

/* Per-level statistics (host copy). */
typedef struct lair_level_stats {
    int64_t n, nnz_A, nc, nnz_R, nnz_P;
    int32_t s_min, s_max;    /* neighbourhood sizes over C-points            */
    double s_mean;
    int64_t n_singular;
} lair_level_stats;

typedef struct lair_hierarchy lair_hierarchy;   /* opaque */

/* Fill the defaults: theta = theta_c = 0.25, ABS, distance 1, one-point P,
 * FP64, omega 1, 25 levels, max_coarse 128, stall 0.9, no block scaling,
 * graph capture on. */
void lair_default_options(lair_strength *s, lair_options *o);

/* Build a hierarchy for A (copied).  cf may be NULL.  On success *out owns
 * all device memory of the hierarchy until lair_free.
 * Errors: EINVAL (bad CSR, non-finite values, bad cf length or values, bad
 * options), ENOMEM, EDEVICE, ESINGULAR (coarsest matrix singular),
 * EUNSUPPORTED (neighbourhood or product row beyond this build's limits). */
lair_status lair_setup(const lair_csr *A, const lair_cf_levels *cf,
                       const lair_strength *s, const lair_options *o,
                       void *stream, lair_hierarchy **out);

/* One V-cycle on device vectors: x <- x + B (b - A x), nrhs interleaved
 * right-hand sides (nrhs in 1, 2, 4, 8, 16, 32).  With block scaling, b is
 * the unscaled right-hand side.  Asynchronous on `stream`. */
lair_status lair_cycle(lair_hierarchy *h, const double *b, double *x,
                       int32_t nrhs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * operation of lair_cycle, x <- x + B (b - A x) on device vectors, with the
 * cycle's work vectors in a fixed device array of the library instead of
 * memory it allocates.  The call allocates nothing (no hipMalloc, no
 * hipFree, no allocating library routine; the kernel profiler must be off,
 * since it creates events).  The array holds LAIR_NOALLOC_MAX_BYTES on every
 * GPU the library runs on, for the life of the process; the first call on a
 * device looks its address up.  The cycle needs, in 256-byte aligned pieces,
 * for every level l four vectors of n_l * nrhs doubles (plus four of floats
 * in LAIR_MIXED), and at level 0 up to two more (block scaling, mixed
 * precision or the F-first ordering); a hierarchy and nrhs whose vectors do
 * not fit give LAIR_EUNSUPPORTED before any device work, leaving x
 * unchanged.  The result is bitwise that of lair_cycle.  Every call on one
 * GPU shares its array, which keeps the last call's contents (the cycle
 * writes every work vector before reading it, so nothing needs clearing):
 * calls that overlap on one GPU, on any streams or hierarchies, race and
 * must not be issued.  Asynchronous on `stream`; the current device's array
 * is used.  Errors otherwise as lair_cycle. */
#define LAIR_NOALLOC_MAX_BYTES (32 << 20)
lair_status lair_cycle_noalloc(lair_hierarchy *h, const double *b, double *x,
                               int32_t nrhs, void *stream);

/* Stationary V-cycle iteration from the given x (device, in/out) until
 * every right-hand side has ||b - A x||_2 <= rtol ||b||_2, or maxit cycles.
 * info may be NULL.  Returns ENOCONV (info filled, x = last iterate) when
 * maxit is reached first. */
lair_status lair_solve(lair_hierarchy *h, const double *b, double *x,
                       int32_t nrhs, double rtol, int32_t maxit,
                       lair_info *info, void *stream);

/* Flexible GMRES(restart) on A x = b with one V-cycle from zero as the
 * right preconditioner: the Krylov solver around the cycle behind the
 * paper's results (Sec. 4; flexible GMRES after Saad, 1993).  Arnoldi by
 * classical Gram-Schmidt applied twice, the least-squares problem by Givens
 * rotations.  Every right-hand side (nrhs in 1, 2, 4, 8, 16, 32, interleaved
 * as for lair_solve) has its own Krylov space; it stops when its residual
 * estimate reaches rtol ||b||_2, and each cycle of `restart` steps (1..64)
 * ends with the true residual, which decides whether to restart.  x
 * (device, in/out) is the initial guess.  One iteration is one Arnoldi step
 * (one V-cycle); info->iters is the largest count over the right-hand
 * sides, info->relres the largest true relative residual at return.  The
 * call allocates 2 restart + 2 device vectors of n x nrhs doubles and
 * returns them to the library's cache.  Single systems only (EUNSUPPORTED
 * for a batch); ENOCONV when maxit is reached first (x = last iterate). */
lair_status lair_solve_fgmres(lair_hierarchy *h, const double *b, double *x,
                              int32_t nrhs, double rtol, int32_t maxit,
                              int32_t restart, lair_info *info, void *stream);

/* Same for the transposed system A^T lam = g with the transposed cycle
 * (pre-relaxation C, F, F on A^T; restriction P^T; interpolation R^T), the
 * exact adjoint of lair_cycle.  Used for gradients. */
lair_status lair_solve_transpose(lair_hierarchy *h, const double *g,
                                 double *lam, int32_t nrhs, double rtol,
                                 int32_t maxit, lair_info *info,
                                 void *stream);

/* One transposed cycle (the adjoint of lair_cycle). */
lair_status lair_cycle_transpose(lair_hierarchy *h, const double *g,
                                 double *lam, int32_t nrhs, void *stream);

/* Batch of independent systems (each one the problem of Sec. 2 on its own).
 * lair_setup_batch builds one hierarchy for the block-diagonal union of the
 * nsys matrices A[0..nsys): system q owns union rows [o_q, o_q + n_q) with
 * o_q = n_0 + ... + n_{q-1}.  Every phase of the setup and of the cycle is
 * one launch over all systems.  Each system follows the single-system rules
 * on its own: it stops coarsening when its size is <= max_coarse, at
 * max_levels, or when its splitting has no C-point or more than stall * n_q
 * of them; a stopped system passes through the remaining levels unchanged
 * (all its points are C-points, R and P are the identity on them and they
 * are not relaxed) and is solved directly at the union's coarsest level,
 * one dense LU per system (at most 4096 rows each).  The CF splittings are
 * the library's own (cf must be NULL or describe the union's levels).
 * The A[q] must all be host arrays or all device arrays (on_device); each
 * is copied.  Errors: as lair_setup, and EINVAL for nsys < 1, mixed
 * locations, a union of 2^31 rows or entries or more, or a member whose
 * rowptr does not run from 0 to nnz or whose columns leave its rows.
 * Only one right-hand side per system (nrhs = 1) is supported on a batch. */
lair_status lair_setup_batch(int32_t nsys, const lair_csr *A, const lair_cf_levels *cf,
                             const lair_strength *s, const lair_options *o, void *stream,
                             lair_hierarchy **out);

/* Stationary iteration x += B (b - A x) on the union (b, x: device vectors
 * of the union's length, system q at rows [o_q, o_q + n_q)), each system
 * stopping on its own when ||b_q - A_q x_q||_2 <= rtol ||b_q||_2; from then
 * on the cycle skips its rows (its x is final).
 * iters[q] and relres[q] (host arrays of nsys entries, may be NULL) return
 * the cycles spent on system q and its final relative residual; info (may
 * be NULL) gets the maximum of both.  ENOCONV when a system has not
 * converged within maxit cycles.  EINVAL for a hierarchy not built by
 * lair_setup_batch. */
lair_status lair_solve_batch(lair_hierarchy *h, const double *b, double *x, double rtol,
                             int32_t maxit, int32_t *iters, double *relres, lair_info *info,
                             void *stream);

/* Replace the diagonal of A (n values; host memory, or device memory when
 * on_device is 1) and rebuild the hierarchy's values on its structure: the
 * strength masks, CF splittings, neighbourhoods and every sparsity pattern
 * are kept (at level 0 they depend only on off-diagonal entries, Sec. 4),
 * while the local solves (Eq. (system)), the interpolation weights, the
 * Galerkin products (Sec. 2.1) and the coarsest factors are recomputed.
 * For a family A(c) = A0 + diag(c) this replaces a full setup when only c
 * changes.  Synchronises `stream`.  Errors: EINVAL (NULL, or a zero or
 * non-finite diagonal entry; the hierarchy is left unchanged),
 * EUNSUPPORTED (block scaling on), ESINGULAR (the hierarchy is then unusable
 * until a successful update). */
lair_status lair_update_diag(lair_hierarchy *h, const double *diag, int32_t on_device,
                             void *stream);

/* Number of systems of a hierarchy (1 for lair_setup), and for a batch the
 * number of levels each system has on its own (levels: nsys entries). */
int32_t lair_num_systems(const lair_hierarchy *h);
lair_status lair_system_levels(const lair_hierarchy *h, int32_t *levels);

/* Size buckets of the local solves (Sec. 3.1: one dense system per
 * C-point).  Systems with S_i <= e[0] are solved one per lane in registers,
 * S_i <= e[1] by teams of 8 lanes, S_i <= e[2] by teams of 16, S_i <= e[3]
 * by teams of 32, larger ones by one wave each.  With e[4] = 1 the first
 * three buckets share one persistent kernel whose blocks take tiles of
 * systems from a queue; with e[4] = 0 each bucket has a kernel of its own.
 * Binning and solving need no host synchronisation.  Every bucket performs
 * the same operations in the same order, so these choices change speed,
 * never results.  By default the library tunes them: the first time the
 * process meets a level shape (precision, size class, mean row length,
 * largest S_i) it times a few candidates on that level and keeps the
 * fastest for the shape.
 * lair_set_local_buckets fixes the choice for every later setup of the
 * process (edges: 5 values with 0 <= e0 <= 4, e0 <= e1 <= 8, e1 <= e2 <= 16,
 * e2 <= e3 <= 32, e4 in {0, 1}, else EINVAL); NULL returns to tuning.  Not
 * thread-safe against concurrent setups.  lair_local_buckets reports the
 * choice a level's local solves used (edges: 5 values; EINVAL for the
 * coarsest level or a level out of range). */
lair_status lair_set_local_buckets(const int32_t *edges);
lair_status lair_local_buckets(const lair_hierarchy *h, int32_t level, int32_t *edges);

/* Number of levels and per-level statistics. */
int32_t lair_num_levels(const lair_hierarchy *h);
lair_status lair_level_stats_get(const lair_hierarchy *h, int32_t level,
                                 lair_level_stats *st);

/* Copy one array of a level to host memory.  `what` selects:
 *   0 A.rowptr (int32, n+1)   1 A.col (int32)    2 A.val (double)
 *   3 cf (int8, n)            4 strength mask (uint8, nnz_A)
 *   5 R.rowptr  6 R.col  7 R.val     8 P.rowptr  9 P.col  10 P.val
 *   11 neighbourhood offsets (int32, nc+1)  12 neighbourhood list (int32)
 *   13 local-solve fallback flags (int8, nc)
 * *bytes is the capacity of host_buf on input and the size needed on
 * output; host_buf may be NULL to query the size.  EINVAL on a bad level or
 * `what`, or when the buffer is too small. */
lair_status lair_export(const lair_hierarchy *h, int32_t level, int32_t what,
                        void *host_buf, int64_t *bytes);

/* Kernel profiler (measurement aid, not part of the method).  Between
 * lair_profile_begin and lair_profile_end every launch whose category is in
 * the comma-separated list `categories` (NULL or "" = all) is bracketed by
 * HIP events recorded on the stream it runs on, and tagged with its
 * algorithmic bytes and flops (the data the operation must read or write at
 * least once).  lair_profile_end waits for those events and writes a JSON
 * object {category: {launches, ms, ms_max, alg_bytes, alg_flops}} into
 * json (capacity *len bytes; *len returns the size needed, json may be NULL
 * to query).  Categories: strength, cf_lists, nbr, local_small, local_wave,
 * local_lstsq, interp, spgemm_count, spgemm_fill, validate, coarse_setup,
 * residual, restrict, interpolate, jacobi, scatter, norm, coarse_solve,
 * cast, spgemm_compact, lump.  Process-wide; not for concurrent use from several host threads. */
lair_status lair_profile_begin(const char *categories);
lair_status lair_profile_end(char *json, int64_t *len);

/* Release a hierarchy (NULL is ignored).  Waits for the device to finish
 * the launches that may still use its memory, which goes back to the
 * library's cache of device blocks. */
void lair_free(lair_hierarchy *h);

/* Return every cached, unused device block to the HIP runtime (after a
 * device synchronisation).  The library keeps released blocks for reuse by
 * later calls on the same stream; this call gives the memory back. */
void lair_trim(void);
/* Device memory of the library in bytes (host variables, may be NULL):
 * *in_use held by hierarchies and calls in progress, *cached released and
 * kept for reuse (lair_trim returns it).  For leak checks: after a failed
 * call the bytes in use are what they were before it.  Allocation failures
 * can be forced for such checks by setting the environment variable
 * LAIR_DEBUG_MAX_BYTES to a positive number of bytes: a request that would
 * raise the bytes in use above it fails with LAIR_ENOMEM. */
void lair_memory(int64_t *in_use, int64_t *cached);
const char *lair_status_string(lair_status s);
const char *lair_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LAIR_H */
