/*
 * mr3.h -- C ABI of an MI355X-native mixed-precision MRRR eigensolver for the
 * real symmetric tridiagonal eigenproblem T z = lambda z.
 *
 * Method: Petschow, Quintana-Orti, Bientinesi, "Improved accuracy and
 * parallelism for MRRR-based eigensolvers -- a mixed precision approach"
 * (arXiv:1304.1864).  Citations below name the paper's sections, algorithm,
 * equations and tables.
 *
 * The problem (Section 1): given the diagonal d[0..n-1] and off-diagonal
 * e[0..n-2] of T, compute eigenvalues lambda_i (the i-th smallest, ascending)
 * and unit eigenvectors z_i for an index set I.  Following the mixed precision
 * scheme of Section 3.1, input and output are in one format (binary_x) and all
 * internal work uses a more precise one (binary_y):
 *   mr3_solve_f32 : x = binary32, y = binary64  (the single/double pairing, Sec. 4.1)
 *   mr3_solve_f64 : x = binary64, y = double-double (FMA-based double-word
 *                   arithmetic; stands in for the paper's software binary128,
 *                   Sec. 4.1 double/quadruple)
 * The solver is Algorithm 1 (MRRR) with the adjustments of Section 3.2:
 * splitting with |e_i| <= eps_x ||T||_1, a definite root representation
 * perturbed by random relative amounts xi = eps_x, eigenvalue bisection on a
 * binary64 copy of each representation, classification with gaptol
 * (1e-5 for f32, 1e-10 for f64), shifts of clusters by the stationary qd
 * transform in y, and Rayleigh quotient iteration with twisted factorizations
 * stopped at ||r|| <= gap * eps_x * sqrt(n) (Sec. 3.2, "Rayleigh quotient
 * iteration").
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * Memory.  d, e, W, Z are DEVICE pointers on the handle's device, owned by
 *   the caller; the library keeps no pointer after returning.  m (the count
 *   of eigenpairs found) is a HOST pointer.  Workspace (the O(p n) working
 *   storage of Sec. 3.3) comes either from the caller, as `work` (device
 *   memory of work_bytes bytes, any alignment, sized with
 *   mr3_workspace_bytes), in which case the call allocates no device memory,
 *   or, with work == NULL, from a per-handle pool that grows on demand and is
 *   released by mr3_destroy.  A work region smaller than the query's value is
 *   accepted down to mr3_workspace_min_bytes: the representation tree is
 *   then walked in groups of clusters whose child representations fit, each
 *   group's subtree finished before the next (Sec. 3.2, "The representation
 *   tree"), and the eigenvectors of a level are computed in rounds.  Below
 *   the minimum the call fails with the position of work_bytes.  The caller
 *   must not touch the region until the call has returned.
 * Layout.  d has length n, e has length n-1 (e may be NULL when n <= 1).
 *   W receives m eigenvalues in ascending order.  Z (column-major, leading
 *   dimension ldz >= max(1, n)) receives the m unit eigenvectors; Z == NULL
 *   computes eigenvalues only.  The sign of each eigenvector is fixed so that
 *   its entry of largest magnitude is positive.
 * Ranges.  MR3_RANGE_ALL: all n eigenpairs.  MR3_RANGE_VALUE: eigenvalues in
 *   the half-open interval [vl, vu).  MR3_RANGE_INDEX: indices il..iu,
 *   1-based, inclusive (the index set I of Section 1).
 * Synchronisation.  All device work is issued on `stream` (a hipStream_t, or
 *   NULL for the null stream).  Calls are synchronous: they return after the
 *   results are complete, because the host sizes every level's launches from
 *   counts it reads back (how many singletons and clusters the
 *   classification found).
 * Errors.  0 on success.  -k: argument k (1-based position in the call) is
 *   invalid (negative n, NULL pointer where one is required, non-finite
 *   input, vl >= vu, il < 1 or iu > n or il > iu + 1, ldz < n, unknown range,
 *   work region too small).
 *   MR3_ERR_NUMERIC (+1): internal numerical failure after every fallback.
 *   MR3_ERR_HIP (+2): a HIP runtime call failed.  MR3_ERR_NO_DEVICE (+3):
 *   no usable GPU.  On a nonzero status the outputs are undefined.
 * Threads.  A handle may be used by one host thread at a time.
 */
#ifndef MR3_H
#define MR3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MR3_OK 0
#define MR3_ERR_NUMERIC 1
#define MR3_ERR_HIP 2
#define MR3_ERR_NO_DEVICE 3
/* gaptol below the lower end of the interval eq. (gaptolinterval) allows,
 * min{1e-3, eps_y sqrt(n) / eps_x} (n of the longest block with wanted
 * eigenvalues), or below 400 * 2^-53, under which the refinement target
 * 1e-2 gaptol comes within 4 ulp of the binary64 interval endpoints.  (A
 * gaptol below the accuracy of eigenvalues approximated on binary64 copies,
 * (k_rr + k_bi) n eps_x, is not refused: those brackets are refined in y.) */
#define MR3_ERR_GAPTOL 4

typedef enum { MR3_RANGE_ALL = 0, MR3_RANGE_VALUE = 1, MR3_RANGE_INDEX = 2 } mr3_range;

typedef struct mr3_handle_s *mr3_handle;

/* Per-problem range of a batched call. */
typedef struct {
    int range;      /* mr3_range */
    double vl, vu;  /* MR3_RANGE_VALUE */
    int64_t il, iu; /* MR3_RANGE_INDEX */
} mr3_range_desc;

/* Tunable parameters (Section 3.2, Section 4.1).  Zero in a field selects the
 * per-precision default given in brackets [f32 path / f64 path]. */
typedef struct {
    double gaptol;         /* classification tolerance, eq. (gaptol interval) [1e-5 / 1e-10] */
    double bisect_rel;     /* relative width of initial eigenvalue intervals [1e-2 * gaptol] */
    double xi;             /* relative size of the root perturbation [eps_x] */
    double k_elg;          /* element-growth bound for accepting a shifted
                              representation, as a multiple of spdiam [10] */
    double k_rs;           /* RQI stopping constant: ||r|| <= k_rs*gap*eps_x*sqrt(n) [1] */
    int max_depth;         /* cap on the depth of the representation tree [6] */
    int rqi_max_iter;      /* RQI iterations before the bisection fallback [10] */
    int lanes_per_eig;     /* bisection lanes per eigenvalue, 1..64: the
                              LDS-staged multisection takes the largest of 1,
                              2, 3, 4, 6, 8, 12, 16, 24, 32, 64 not above it,
                              the per-lane kernel the largest power of two;
                              0 = from the tuning table, else the size */
    unsigned long long seed; /* seed of the counter-based perturbation generator [0x5eed] */
    /* fault injection (tests): force the bisection fallback of RQI for every
     * eigenvector; reject every candidate shift so the least-growth candidate
     * is used */
    int force_rqi_fallback;
    int force_best_candidate;
    /* 1: time every kernel launch with HIP events recorded on the launch
     * stream; the per-stage totals appear in mr3_stats */
    int profile;
    int points_per_lane;   /* bisection points per lane and pass: 1, 2 or 4;
                              0 = chosen with lanes_per_eig from the size */
    double gaptol_abs;     /* splitting by absolute gaps (Sec. 2, "Classification
                              of the eigenvalues"): neighbours whose gap is at
                              least gaptol_abs * spdiam are separated whatever
                              their relative gap; 0 = off [0] */
    int initial;           /* initial eigenvalue approximations of a root whose
                              whole spectrum is wanted (Sec. 4.1):
                              MR3_INITIAL_BISECTION, or MR3_INITIAL_DQDS for the
                              sequential dqds algorithm, one lane per root of at
                              most MR3_DQDS_MAX_N rows (larger roots and subsets
                              use bisection).  The dqds values are checked with
                              Sturm counts and refined by bisection like any
                              other bracket [MR3_INITIAL_BISECTION] */
    int refine_ends;       /* 1: before a cluster's shift is chosen, refine its
                              two extreme eigenvalues by bisection in y to
                              binary64 resolution (Sec. 3.2, footnote on the
                              refinement of extreme eigenvalues prior to
                              selecting shifts); candidate shifts may then come
                              as close to the cluster as those brackets allow,
                              and their inertia follows from them [0] */
    int force_resort;      /* fault injection (tests): reverse every problem's
                              eigenvalues and eigenvectors on the device before
                              the ascending-order check, so that the host-side
                              reordering runs */
    int derive_lld;        /* 1: the e-representation without cached derived
                              data (Sec. 3.2, "Choice of representations"): a
                              tree node keeps only its d in y (and binary64
                              copies); lld_i = e_i^2 / d_i is formed from the
                              block's off-diagonals, stored once, wherever rows
                              are read in y, with the bits the stored value
                              would have.  Results are identical; each node row
                              takes 16 (FP64) or 8 (FP32) bytes less, and the
                              sweeps and counts in y form one quotient per row
                              they load [0] */
} mr3_params;

#define MR3_INITIAL_BISECTION 0
#define MR3_INITIAL_DQDS 1
#define MR3_DQDS_MAX_N 4096

/* Diagnostics of the last solve on a handle (Section 4.2 reports d_max and
 * the clustering rho = largest cluster / n). */
typedef struct {
    int64_t n_eigenpairs;     /* m of the last call (summed over a batch) */
    int64_t n_blocks;         /* irreducible blocks after splitting */
    int d_max;                /* depth of the deepest representation-tree node */
    int64_t n_clusters;       /* clusters processed (all levels) */
    int64_t largest_cluster;  /* size of the largest cluster */
    int64_t n_rqi_iters;      /* RQI iterations summed over eigenvectors */
    int64_t n_fallbacks;      /* eigenvectors that needed the bisection fallback */
    int64_t n_best_candidate; /* shifts accepted as least-growth candidate */
    /* with mr3_params.profile = 1: device time (ms) and launch count per
     * stage, indexed by MR3_STAGE_* */
    double stage_ms[8];
    int64_t stage_launches[8];
    /* algorithmic work of the last solve: Sturm-count row steps that plain
     * bisection needs for the final intervals, and row steps of twisted
     * sweeps (pre-pass and RQI iterations) */
    double bisect_row_steps;
    double rqi_row_steps;
    double twist_row_steps;
    int64_t n_dqds_roots;     /* roots whose initial eigenvalues came from dqds */
    int64_t dqds_transforms;  /* shifted qd transforms summed over those roots */
    int64_t n_sliced_roots;   /* roots whose multisection started from spectrum
                                 slicing (shared Sturm counts at equally spaced
                                 points) */
    int n_singleton_first_levels; /* tree levels whose singleton work was
                                     issued before their cluster work (the
                                     throughput-bound order of large batches) */
    int64_t n_y_refined;      /* eigenvalue brackets refined by bisection in y
                                 because the binary64 copy of their node does
                                 not resolve gaptol (Sec. 3.2, "Arithmetic
                                 used to approximate eigenvalues") */
    int64_t n_resorted;       /* problems whose eigenpairs came out of order
                                 and were reordered on the host */
    /* the largest multisection launch of each kind in the last solve, indexed
     * by MR3_TUNE_ROOT / MR3_TUNE_CHILD: eigenvalues it bisected, the mean row
     * count of their nodes, and the lanes per eigenvalue it took (the key and
     * the result of a look-up in the tuning table below; 0 when none ran) */
    int64_t bisect_count[2];
    int64_t bisect_rows[2];
    int bisect_lanes[2];
} mr3_stats;

/* stage indices of mr3_stats.stage_ms */
#define MR3_STAGE_PREP 0     /* preprocessing, root representation, products */
#define MR3_STAGE_BISECT 1   /* multisection on Sturm counts (k_bisect) */
#define MR3_STAGE_CLASSIFY 2 /* classification and list compaction */
#define MR3_STAGE_RQI 3      /* twisted-factorization RQI (k_rqi) */
#define MR3_STAGE_ZOUT 4     /* eigenvector output (k_zout) */
#define MR3_STAGE_CHILD 5    /* cluster shifts (k_child_select, k_child_rep) */
#define MR3_STAGE_CBISECT 6  /* multisection of child eigenvalues (k_bisect) */
#define MR3_STAGE_VERIFY 7   /* check of child brackets in working precision (k_verify) */

/* Create a handle on HIP device `device`.  Fails with MR3_ERR_NO_DEVICE if it
 * does not exist. */
int mr3_create(mr3_handle *h, int device);
/* Release the handle and its workspace pool. */
int mr3_destroy(mr3_handle h);
/* Fill *p with the defaults for `precision` (32 or 64). */
int mr3_default_params(mr3_params *p, int precision);
/* Replace the handle's parameters (copied).  NULL restores the defaults. */
int mr3_set_params(mr3_handle h, const mr3_params *p);
/* Diagnostics of the last solve. */
int mr3_get_stats(mr3_handle h, mr3_stats *s);

/* Multisection shapes measured on the device (the autotuner's table).  The
 * eigenvalue intervals of a level are refined by multisection (Sec. 2,
 * Alg. 1: bisection to classify and to start RQI) with L lanes per
 * eigenvalue: each pass counts at L points and gains log2(L + 1) bits, so a
 * larger L costs more Sturm counts but fewer dependent passes.  A launch over
 * `count` eigenvalues whose nodes have on average `rows` rows takes `lanes`
 * from the first entry whose stage and precision match and whose ranges hold
 * count and rows; with no such entry a size rule is used, and a nonzero
 * mr3_params.lanes_per_eig overrides both.  A handle starts with the table
 * the library was built with, which the package's tuner writes from timed
 * runs of this kind on gfx950. */
#define MR3_TUNE_ROOT 0  /* root eigenvalues (stage MR3_STAGE_BISECT) */
#define MR3_TUNE_CHILD 1 /* members of clusters in their child nodes (MR3_STAGE_CBISECT) */
typedef struct {
    int stage;                  /* MR3_TUNE_ROOT or MR3_TUNE_CHILD */
    int precision;              /* 32 or 64: I/O precision of the solve */
    int64_t count_lo, count_hi; /* eigenvalues in the launch: count_lo <= count < count_hi */
    int64_t rows_lo, rows_hi;   /* mean rows of their nodes: rows_lo <= rows < rows_hi */
    int lanes;                  /* lanes per eigenvalue: 1, 2, 3, 4, 6, 8, 12, 16, 24, 32 or 64 */
    int reserved;               /* 0 */
} mr3_tune_entry;

/* Replace the handle's table by a copy of t[0 .. count): count 0 leaves no
 * table (size rules only); t NULL with count < 0 restores the built-in table.
 * Returns -1 for a null handle, -2 (table unchanged) for an entry with an
 * unknown stage or precision, an empty range or a lanes value not listed
 * above. */
int mr3_set_tuning(mr3_handle h, const mr3_tune_entry *t, int count);

/* Copy up to `cap` entries of the handle's table to t (t may be NULL when cap
 * is 0).  Returns the number of entries in the table, -1 for a null handle. */
int mr3_get_tuning(mr3_handle h, mr3_tune_entry *t, int cap);

/* Lanes per eigenvalue that a multisection launch of this stage, precision,
 * eigenvalue count and mean node rows takes from the handle's override or
 * table; 0 when neither applies (the size rule decides).  -1 for a null
 * handle, -2 for an unknown stage or precision. */
int mr3_bisect_lanes(mr3_handle h, int stage, int precision, int64_t count, int64_t rows);

/* Single problem, FP32 input/output with binary64 internal arithmetic
 * (Section 4.1, single/double).  Arguments (1-based positions, used in the
 * -k error codes): 1 h, 2 n, 3 d, 4 e, 5 range, 6 vl, 7 vu, 8 il, 9 iu,
 * 10 m, 11 W, 12 Z, 13 ldz, 14 work (device, or NULL for the handle's pool),
 * 15 work_bytes, 16 stream. */
int mr3_solve_f32(mr3_handle h, int64_t n, const float *d, const float *e, int range,
                  double vl, double vu, int64_t il, int64_t iu, int64_t *m, float *W,
                  float *Z, int64_t ldz, void *work, size_t work_bytes, void *stream);

/* Single problem, FP64 input/output with double-double internal arithmetic
 * (Section 4.1, double/quadruple, with double-double as y).  Same arguments. */
int mr3_solve_f64(mr3_handle h, int64_t n, const double *d, const double *e, int range,
                  double vl, double vu, int64_t il, int64_t iu, int64_t *m, double *W,
                  double *Z, int64_t ldz, void *work, size_t work_bytes, void *stream);

/* Device bytes of a work region with which a single solve of order n runs at
 * full speed (the whole root level's eigenvectors in one round, and up to
 * 512 clusters per level expanded at once), for any matrix of that order:
 * range is an mr3_range, k_max bounds the wanted eigenpairs of INDEX and
 * VALUE ranges (<= 0: unknown, taken as n), precision is 32 or 64.  The size
 * follows the handle's parameters (depth cap, dqds option); h may be NULL for
 * the defaults.  Returns 0 for invalid arguments or n = 0 (no work region
 * needed). */
size_t mr3_workspace_bytes(mr3_handle h, int64_t n, int range, int64_t k_max, int precision);

/* The smallest work region with which every single solve of order n runs
 * (arguments as for mr3_workspace_bytes): the roots plus one child
 * representation per tree level, and eigenvectors in rounds of one chunk of
 * 32.  Any size between the two is accepted and runs at a speed between. */
size_t mr3_workspace_min_bytes(mr3_handle h, int64_t n, int range, int64_t k_max, int precision);

/* The same for a batched call of `count` problems with orders n[count] and
 * ranges[count] (host; NULL = all pairs). */
size_t mr3_workspace_bytes_batched(mr3_handle h, int64_t count, int precision, const int64_t *n,
                                   const mr3_range_desc *ranges);

/* Many independent problems of one precision in one pass of the pipeline
 * (every stage is a single launch over all problems).
 * Arguments: 1 h, 2 count, 3 precision (32 or 64), 4 n[count] (host),
 * 5 de_off[count] (host; problem p reads d + de_off[p] and e + de_off[p]),
 * 6 d, 7 e (device, float or double per precision), 8 ranges[count] (host,
 * NULL = all), 9 m[count] (host, output), 10 W (device), 11 w_off[count]
 * (host), 12 Z (device, may be NULL), 13 z_off[count] (host), 14 ldz[count]
 * (host), 15 work (device, or NULL for the handle's pool), 16 work_bytes,
 * 17 stream. */
int mr3_solve_batched(mr3_handle h, int64_t count, int precision, const int64_t *n,
                      const int64_t *de_off, const void *d, const void *e,
                      const mr3_range_desc *ranges, int64_t *m, void *W, const int64_t *w_off,
                      void *Z, const int64_t *z_off, const int64_t *ldz, void *work,
                      size_t work_bytes, void *stream);

/* ---- Single solve that allocates nothing ----
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it).  The same solve as
 * mr3_solve_f32 (precision 32) or mr3_solve_f64 (precision 64) with the work
 * region taken from a static device array of the library,
 * MR3_NOALLOC_SCRATCH_BYTES long, one per GPU, allocated when the library's
 * code object is loaded on that GPU and held until the process ends; its
 * device address is resolved once per device by mr3_create.  The call
 * allocates no device or pinned host memory.  Every call on a GPU shares that
 * GPU's array (within one process; each process has its own copy), which
 * keeps the last call's contents, so calls that overlap on one GPU, from
 * several host threads or handles, race: serialise them.  Arguments: 1 h, 2 precision (32 or 64), 3 n (at most
 * MR3_NOALLOC_MAX_N), 4 d, 5 e, 6 range, 7 vl, 8 vu, 9 il, 10 iu, 11 m, 12 W,
 * 13 Z, 14 ldz, 15 stream, as for mr3_solve_f32 / mr3_solve_f64.  Errors as
 * there; n above MR3_NOALLOC_MAX_N returns -3. */
#define MR3_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
#define MR3_NOALLOC_MAX_N 16384
int mr3_solve_noalloc(mr3_handle h, int precision, int64_t n, const void *d, const void *e,
                      int range, double vl, double vu, int64_t il, int64_t iu, int64_t *m, void *W,
                      void *Z, int64_t ldz, void *stream);

/* ---- Dense symmetric and Hermitian eigenproblems (Section 4.2, Fig. 3) ----
 *
 * The pipeline of the paper's dense experiments: reduce A to tridiagonal
 * form A = Q T Q^H (Householder reduction, rocSOLVER sytrd / hetrd), compute
 * the wanted eigenpairs of T with this library's solver of the same I/O
 * precision (mixed precision inside), and back-transform the eigenvectors
 * Z := Q Z (rocSOLVER ormtr / unmtr).  T is real symmetric in every case:
 * the Hermitian reduction leaves a real tridiagonal.
 *
 * A: n x n, column-major, leading dimension lda >= max(1, n), device; only
 * its lower triangle is read, and the call overwrites it with the reflectors.
 * range, vl, vu, il, iu, m: as for mr3_solve_f32.  W: m eigenvalues,
 * ascending, device, real (float for _f32 and _c64, double otherwise).  Z:
 * n x m eigenvectors, column-major, leading dimension ldz >= max(1, n),
 * device, of A's element type (a complex number is two reals, real part
 * first: two floats for _c64, two doubles for _c128), or NULL for
 * eigenvalues only.  stream: as for the solves.
 * Synchronous, like the other calls.  These entry points allocate: the
 * tridiagonal's d, e and the reflector scalars (3n elements), for the complex
 * forms the real eigenvectors of T (n m reals), the solver's work through the
 * handle's pool, and rocSOLVER's own workspace.
 * Returns MR3_OK, the solver's error codes, MR3_ERR_HIP for a failed
 * reduction or back-transformation, or -k for an invalid argument k
 * (1 h, 2 n, 3 A, 4 lda, 5 range, 6 vl, 7 vu, 8 il, 9 iu, 10 m, 11 W, 12 Z,
 * 13 ldz, 14 stream); n above 2^31 - 1 is argument 2's error. */
int mr3_dense_f32(mr3_handle h, int64_t n, float *A, int64_t lda, int range, double vl,
                  double vu, int64_t il, int64_t iu, int64_t *m, float *W, float *Z,
                  int64_t ldz, void *stream);
int mr3_dense_f64(mr3_handle h, int64_t n, double *A, int64_t lda, int range, double vl,
                  double vu, int64_t il, int64_t iu, int64_t *m, double *W, double *Z,
                  int64_t ldz, void *stream);
int mr3_dense_c64(mr3_handle h, int64_t n, void *A, int64_t lda, int range, double vl,
                  double vu, int64_t il, int64_t iu, int64_t *m, float *W, void *Z,
                  int64_t ldz, void *stream);
int mr3_dense_c128(mr3_handle h, int64_t n, void *A, int64_t lda, int range, double vl,
                   double vu, int64_t il, int64_t iu, int64_t *m, double *W, void *Z,
                   int64_t ldz, void *stream);

/* Verification (not part of a solve; Section 1, eq. (1)).  For the FP64
 * eigenpairs (W, Z) of the FP64 tridiagonal (d, e), all device pointers:
 * orth_out[0] = max_{i != j} |z_i^T z_j| and orth_out[1] = max_i |z_i^T z_i - 1|,
 * computed from Z^T Z with FP64 matrix-core (MFMA) tiles; resid_out[0] =
 * max_i ||T z_i - lambda_i z_i||_1 / ||T||_1.  Host outputs.  Arguments: 1 h,
 * 2 n, 3 m, 4 d, 5 e, 6 W, 7 Z, 8 ldz, 9 orth_out[2], 10 resid_out[1],
 * 11 stream. */
int mr3_check_f64(mr3_handle h, int64_t n, int64_t m, const double *d, const double *e,
                  const double *W, const double *Z, int64_t ldz, double *orth_out,
                  double *resid_out, void *stream);

/* ---- Serving: continuous batching of independent requests ----
 *
 * A server runs max_inflight worker slots on the handle's device, each with
 * its own solver handle (the caller's for slot 0, copies of its parameters
 * for the others) and stream.  Requests queue in arrival order; an idle slot
 * takes the oldest request and the later queued requests of the same
 * precision (at most max_batch) whose estimated work regions fit the largest
 * free part of the server's memory, and solves them as one batch, exactly
 * like mr3_solve_batched.  Requests that arrive while batches run are
 * admitted as slots and memory free up, so batches overlap on the device, FP32
 * and FP64 ones included.  The server allocates one device arena of
 * hbm_budget_bytes at creation and runs every batch on a region of it sized by
 * mr3_workspace_bytes_batched: device use never exceeds the budget and the
 * solves allocate nothing.  A request whose region does not fit waits for a
 * batch to end; with nothing else running it gets the whole arena.  The
 * paper's eigenpairs are independent (Section 3.1), so a batch's results
 * equal those of solving each request alone, to the gates. */
typedef struct mr3_server_s *mr3_server;

typedef struct {
    int precision;        /* 32 or 64: element type of d, e, W, Z */
    int64_t n;            /* order of T */
    const void *d;        /* device, n elements */
    const void *e;        /* device, n-1 elements (may be NULL for n <= 1) */
    mr3_range_desc range; /* which eigenpairs */
    void *W;              /* device output, room for every requested eigenvalue */
    void *Z;              /* device output, column-major ldz x m, or NULL */
    int64_t ldz;
    void *stream;         /* hipStream_t on which d and e are produced (NULL: the
                             null stream); the solve starts after the work
                             queued there before mr3_server_submit */
} mr3_request;

typedef struct {
    int status;         /* 0, or the error code of the batch solve */
    int64_t m;          /* eigenpairs computed */
    double submit_ms;   /* host steady clock (ms) at submit */
    double start_ms;    /* ... when its batch was launched */
    double done_ms;     /* ... when its batch had completed on the device */
    int64_t batch_id;   /* batches are numbered from 0 in the order they form */
    int batch_size;     /* requests in that batch */
    int slot;           /* worker slot that ran the batch */
} mr3_result;

/* Work region (device bytes) a request of order n with k wanted eigenpairs is
 * budgeted at: mr3_workspace_bytes of the request alone with the default
 * parameters (k >= n: all pairs). */
size_t mr3_request_bytes(int64_t n, int64_t k, int precision);

/* Create a server that takes over handle h (the caller must not use h until
 * mr3_server_destroy returns), with two worker slots.  Arguments: 1 s
 * (output), 2 h, 3 hbm_budget_bytes (> 0; allocated on the device here), 4
 * max_batch (>= 1).  MR3_ERR_HIP if the arena or the slots' streams cannot be
 * created. */
int mr3_server_create(mr3_server *s, mr3_handle h, size_t hbm_budget_bytes, int max_batch);

/* The same with 5 max_inflight worker slots (1 to 8). */
int mr3_server_create_ex(mr3_server *s, mr3_handle h, size_t hbm_budget_bytes, int max_batch,
                         int max_inflight);

/* Host-side scheduler tests: batches go to fn(ctx, count, reqs, m) instead of
 * the device solver (called from max_inflight worker threads); fn returns a
 * status and fills m[count].  No device memory is allocated; a request is
 * budgeted at mr3_request_bytes. */
typedef int (*mr3_executor_fn)(void *ctx, int64_t count, const mr3_request *reqs, int64_t *m);
int mr3_server_create_with_executor(mr3_server *s, mr3_executor_fn fn, void *ctx,
                                    size_t hbm_budget_bytes, int max_batch, int max_inflight);

/* Queue a request (copied; its device buffers must stay valid until the
 * request completes).  Returns a ticket.  Arguments: 1 s, 2 r, 3 ticket.
 * Errors: -2 r NULL or invalid (precision, n, pointers, range, ldz); -3 the
 * request cannot run even alone in the whole budget (its minimum work
 * region, mr3_workspace_min_bytes, exceeds it); -4 ticket NULL;
 * MR3_ERR_HIP if the ordering event cannot be recorded on r->stream. */
int mr3_server_submit(mr3_server s, const mr3_request *r, uint64_t *ticket);

/* *done = 1 once the request's batch has completed, else 0; -2 unknown ticket. */
int mr3_server_poll(mr3_server s, uint64_t ticket, int *done);

/* Block until the request has completed, copy its result to *out (may be
 * NULL) and release the ticket.  Returns the request's status; -2 for an
 * unknown ticket or one another thread is already waiting for. */
int mr3_server_wait(mr3_server s, uint64_t ticket, mr3_result *out);

/* Finish every queued request, stop the workers and free the server and its
 * arena (not the handle, which the caller may use again). */
int mr3_server_destroy(mr3_server s);

/* Library version string. */
const char *mr3_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MR3_H */
