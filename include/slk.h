/*
 * slk.h -- C ABI of libslk, an MI355X (gfx950) implementation of the bound-optimizer
 * iteration of Scalable Laplacian K-modes (SLK-BO; Ziko, Granger, Ben Ayed, NeurIPS 2018).
 *
 * The calls follow the paper's problem statement: points X = {x_p in R^D} and a number
 * of clusters L (Section 1, Eq. (1)); a Laplacian weight lambda (Eq. (1)); the Gaussian
 * kernel k(x, y) = exp(-||x - y||^2 / (2 sigma^2)) and the binary kNN affinity with its
 * sigma^2 estimator (Section 4.2); initial modes (Algorithm 1, input); outputs Z and the
 * modes {m_l} (Algorithm 1, output).
 *
 * Conventions shared by every call:
 *  - Pointers are DEVICE pointers unless the parameter name ends in `_host`.
 *  - Arrays are dense, row-major, contiguous: X is n x d float32, Z is n x L float32,
 *    labels are n int32, kNN lists are n x k.
 *  - Point indices (modes, labels' rows, kNN lists, CSR columns) are 0-based and always
 *    in the caller's original point order; an internal locality permutation is hidden.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is stream-ordered.  A call
 *    with a `_host` output synchronises `stream` before it returns; device outputs are
 *    complete when the stream reaches the call's end.
 *  - The caller owns every array it passes in; the library never frees caller memory.
 *    Graph handles are owned by the library until slk_graph_destroy.  Temporary device
 *    memory stays with the library for later calls on the same device: slk_fit, slk_assign,
 *    slk_fit_ms and slk_energy (which synchronise their stream before returning) carve theirs
 *    from one kept block per concurrent call, as large as the largest such call needed; the
 *    other calls take it from a stream-ordered pool that keeps up to 4 GiB of freed memory.
 *    slk_pool_trim releases both.
 *  - Errors are returned as slk_status; no exception or abort crosses the ABI.  Arguments
 *    are validated before any launch; on a non-OK status the outputs are unspecified and
 *    slk_last_error() describes the failure (thread-local text, valid until the next call
 *    on the same thread).
 *  - Results are deterministic: the same inputs and parameters give bit-identical
 *    outputs (all reductions run in a fixed order).
 *  - Limits: 2 <= n < 2^31, d >= 1, 1 <= k <= 64, 1 <= L <= 256, n * L' < 2^30 where L' is L
 *    rounded up to a multiple of 4, total CSR entries < 2^31.
 */
#ifndef SLK_H_
#define SLK_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLK_OK = 0,
  SLK_ERR_INVALID_ARG = 1,   /* a size, pointer or parameter is out of range          */
  SLK_ERR_OUT_OF_MEMORY = 2, /* a device or pinned host allocation failed             */
  SLK_ERR_DEVICE = 3,        /* a HIP runtime call or kernel launch failed            */
  SLK_ERR_NUMERIC = 4,       /* the relaxed bound became NaN or infinite              */
  SLK_ERR_UNSUPPORTED = 5    /* a valid request the library does not implement         */
} slk_status;

/* Precision of the points used by the distance computations. */
typedef enum {
  SLK_PREC_FP32 = 0,  /* X as given (float32)                                            */
  SLK_PREC_BF16 = 1,  /* X rounded to bfloat16 once; all distances use the rounded points */
  SLK_PREC_BF16X = 2  /* unary distances as a bf16 MFMA contraction with FP32 accumulation of
                         X split into two bf16 terms (hi + lo, tile-centred); X itself is not
                         rounded; the kNN graph is built as for FP32 (its candidates are bf16
                         MFMA products already).  For fits, assignments, slk_unary, slk_predict. */
} slk_precision;

/* Candidate search used by slk_build_knn. */
typedef enum {
  SLK_KNN_AUTO = 0,  /* exact FP64 brute force for small n*n*d, else MFMA candidates     */
  SLK_KNN_EXACT = 1, /* every distance in FP64                                           */
  SLK_KNN_MFMA = 2   /* bf16 MFMA Gram candidates + FP64 re-rank + certificate           */
} slk_knn_method;

typedef struct slk_graph slk_graph; /* opaque: device-resident kNN lists, CSR, sigma^2 */

typedef struct {
  int32_t k;          /* k_n, neighbours per point (Section 4.2); 1 <= k <= 64, k < n      */
  int32_t reorder;    /* 1: relabel points internally for neighbour locality (BFS order)   */
  int32_t candidates; /* MFMA path: candidates kept per row before the exact re-rank
                         (0 = automatic: max(2k, 32); clamped to [k, 64])                             */
  slk_knn_method method;
  slk_precision prec;
} slk_knn_opts;

typedef struct {
  int64_t n;
  int32_t k;            /* 0 for a graph imported from CSR                                 */
  int32_t reordered;    /* 1 if an internal locality permutation is in use                 */
  int64_t nnz;          /* stored CSR entries (ordered pairs)                               */
  int32_t max_degree;
  int32_t min_degree;
  double sigma2;        /* kNN bandwidth estimate (<= 0 if unknown, e.g. CSR import)       */
  int64_t rows_certified;  /* MFMA path: rows whose top-k the error bound certified        */
  int64_t rows_fallback;   /* MFMA path: rows recomputed by the exact FP64 search          */
} slk_graph_info_t;

/* Fill *opts with defaults: k = 10, reorder = 0, candidates = 0, AUTO, FP32. */
slk_status slk_knn_opts_default(slk_knn_opts* opts);

/*
 * Build the kNN affinity of Section 4.2 from the points.
 *  x      : n x d float32 points (device).
 *  For every p the k nearest q != p under the Euclidean distance are found, ordered by
 *  (squared distance, index) -- ties go to the smaller index.  The reported squared
 *  distances are the FP64 sum over j = 0..d-1, in order, of (x_pj - x_qj)^2 with every
 *  subtraction, square and addition rounded separately.  The binary affinity
 *  w_pq = 1 iff q in N_p or p in N_q (no self-loops) is stored as CSR, and
 *  sigma^2 = (1 / (n k)) sum_p sum_{q in N_p} ||x_p - x_q||^2  (Section 4.2).
 *  On success *g_out receives a new handle (release with slk_graph_destroy).
 *  Synchronises `stream`.
 */
slk_status slk_build_knn(const float* x, int64_t n, int32_t d, const slk_knn_opts* opts,
                         void* stream, slk_graph** g_out);

/* One problem of slk_build_knn_batched. */
typedef struct {
  const float* x;     /* n x d float32 points (device)                                      */
  int64_t n;
  int32_t d;
  int32_t reserved;   /* 0                                                                  */
  slk_knn_opts opts;
} slk_knn_item;

/*
 * slk_build_knn for several independent problems at once (the batched form's graph build):
 * graphs_out[i] receives the graph of items[i], identical to slk_build_knn's for the same
 * arguments (lists, distances, CSR, sigma^2).  The problems that take the exact search (method
 * EXACT, or AUTO with n^2 d <= 4e9) share ONE launch of that search, each problem keeping its own
 * work-groups; the others are built one by one.  On any failure no graph is returned (every
 * graphs_out[i] is NULL).  Synchronises `stream`.
 */
slk_status slk_build_knn_batched(const slk_knn_item* items, int32_t count, void* stream, slk_graph** graphs_out);

/*
 * Build the graph from given kNN lists (device): knn_idx n x k int32 (original indices,
 * each row free of p itself), knn_d2 n x k float64 (their squared distances, used only
 * for sigma^2; may be NULL, then sigma^2 is unknown).  Same symmetrisation as above.
 * Synchronises `stream`.
 */
slk_status slk_graph_from_knn(int64_t n, int32_t k, const int32_t* knn_idx, const double* knn_d2,
                              int32_t reorder, void* stream, slk_graph** g_out);

/*
 * Import a binary affinity given as CSR (device arrays): row_ptr n+1 int32 (row_ptr[0] = 0,
 * non-decreasing, row_ptr[n] = nnz), col_idx nnz int32 in [0, n).  The matrix should be
 * symmetric for the bound of Proposition 1 to hold; it is used as given (duplicates count
 * twice, self-loops act as a diagonal shift).  sigma2_hint is stored as the graph's sigma^2
 * (<= 0 = unknown).  The arrays are copied.  Synchronises `stream`.
 */
slk_status slk_graph_from_csr(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                              double sigma2_hint, int32_t reorder, void* stream, slk_graph** g_out);

/* Sizes and statistics of a graph (host struct). */
slk_status slk_graph_info(const slk_graph* g, slk_graph_info_t* info_host);

/*
 * Copy the graph out, in the original point order (device outputs, any may be NULL):
 * row_ptr n+1 int32, col_idx nnz int32 (columns sorted within each row), knn_idx n x k int32,
 * knn_d2 n x k float64 (kNN outputs need a graph built from points or kNN lists).
 * perm n int32: perm[i] = original index of internal row i (identity if not reordered).
 * Synchronises `stream`.
 */
slk_status slk_graph_export(const slk_graph* g, int32_t* row_ptr, int32_t* col_idx, int32_t* knn_idx,
                            double* knn_d2, int32_t* perm, void* stream);

void slk_graph_destroy(slk_graph* g);

typedef struct {
  double lambda;          /* Laplacian weight (Eq. (1)); >= 0                                   */
  double sigma2;          /* Gaussian bandwidth; <= 0 uses the graph's estimate (Section 4.2)   */
  double delta;           /* diagonal shift K + delta I (footnote to Proposition 1); >= 0       */
  double bound_tol;       /* inner stop: |R(Z^{i+1}) - R(Z^i)| <= tol |R(Z^i)|                  */
  int32_t max_outer;      /* cap on mode updates (Algorithm 1, outer loop)                      */
  int32_t max_inner;      /* cap on z-updates per outer iteration                               */
  int32_t fixed_inner;    /* > 0: run exactly this many z-updates, no convergence test          */
  int32_t pairwise_scale; /* 1: z = softmax(a + lambda b) as in Eq. (8); 2: softmax(a + 2 lambda b),
                             the exact minimiser for Eq. (2) as printed                          */
  slk_precision prec;     /* precision of X in the unary distances                              */
  int32_t final_pass;     /* 0: for 8 < L <= 64 the z-update expected to end the inner loop also
                             writes the labels and mode candidates of its input, and a separate
                             final pass runs only if another pass ended it; 1: always the separate
                             final pass.  The results are identical.                            */
} slk_params;

typedef struct {
  int32_t outer_iters;        /* outer iterations run                                       */
  int32_t inner_iters_total;  /* z-updates run over all outer iterations                    */
  int32_t inner_iters_last;   /* z-updates of the last outer iteration                      */
  int32_t converged;          /* fit: modes unchanged; assign: bound settled (or fixed count) */
  int32_t n_distinct_modes;
  int32_t final_passes;       /* outer iterations that ran a separate final pass             */
  double energy;              /* E(l, M) of Eq. (1) at the hard labels, unary term from FP32 A  */
  double energy_fp64;         /* the same with the unary term recomputed in FP64 from X         */
  double bound;               /* relaxed bound R(Z^i) of the last z-update's input              */
  int64_t cut;                /* ordered neighbour pairs with different labels                  */
} slk_result;

/* Fill *p with defaults: lambda 1, sigma2 0 (graph), delta 0, tol 1e-8, max_outer 20,
   max_inner 1000, fixed_inner 0, pairwise_scale 1, FP32. */
slk_status slk_params_default(slk_params* p);

/*
 * One outer iteration of Algorithm 1 with the modes fixed (its z-update block):
 *   a_pl = k(x_p, m_l)                                  (Eq. (6a))
 *   z_p^0 = softmax(a_p)                                (Algorithm 1, initialisation)
 *   repeat: b_p = sum_q w_pq z_q^i (+ delta z_p^i)      (Eq. (6b))
 *           z_p^{i+1} = softmax(a_p + lambda b_p)       (Eq. (8)), all p in parallel
 *   until the relaxed bound settles (see slk_params.bound_tol) or max_inner/fixed_inner.
 *   Then: labels l_p = argmax_l (a_p + lambda b_p)_l (ties to the smaller l) and the
 *   byproduct modes m_l = x_q, q = argmax_q z_ql (Eq. (11)), ranked by the log-odds
 *   log(z_ql / (1 - z_ql)) computed from the logits, ties to the smaller index.
 *  x            : n x d float32 (device), the points the graph was built on.
 *  modes_host   : L distinct int32 point indices (host).
 *  z_out        : n x L float32 (device) receives the last z-update.
 *  labels_out   : n int32 (device, may be NULL).
 *  modes_next_host : L int32 (host, may be NULL) receives the byproduct modes.
 *  bound_trace_host : (host, may be NULL) receives the relaxed bound R(Z^i) of every
 *                 z-update, up to trace_cap values.
 *  res_host     : summary (host, may be NULL).  Synchronises `stream`.
 */
slk_status slk_assign(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L,
                      const int32_t* modes_host, const slk_params* p, void* stream, float* z_out,
                      int32_t* labels_out, int32_t* modes_next_host, double* bound_trace_host,
                      int32_t trace_cap, slk_result* res_host);

/*
 * SLK-BO (Algorithm 1): alternate slk_assign's z-update block with the byproduct mode
 * update until the modes do not change (Section 3) or max_outer.  Z restarts from
 * softmax(a) in every outer iteration, as in Algorithm 1.
 *  init_modes_host : L distinct int32 indices (host).
 *  z_out, labels_out : as in slk_assign, for the last outer iteration.
 *  modes_out_host  : L int32 (host) final modes.
 *  res_host        : summary (host, may be NULL); energy is E(l, M) at the last labels and
 *                    the modes that produced them.  Synchronises `stream`.
 */
slk_status slk_fit(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L,
                   const int32_t* init_modes_host, const slk_params* p, void* stream, float* z_out,
                   int32_t* labels_out, int32_t* modes_out_host, slk_result* res_host);

typedef struct {
  double energy;       /* E(l, M), Eq. (1) with Eq. (3), unary term from FP32 distances      */
  double energy_fp64;  /* unary term recomputed in FP64                                     */
  double bound;        /* relaxed bound R(Z) if z was given, else 0                          */
  int64_t cut;         /* ordered pairs (p, q), w_pq = 1, l_p != l_q                          */
} slk_energy_out;

/*
 * Discrete energy of Eq. (1) for hard labels (device, n int32 in [0, L)) and modes
 * (host, L int32): E = -sum_p k(x_p, m_{l_p}) + lambda * cut.  If z (device, n x L) is
 * given, also the relaxed bound  R(Z) = sum_p [z_p.log z_p - z_p.a_p - (lambda/2) z_p.b_p],
 * b = (W + delta I) Z.  sigma2 <= 0 uses the graph's estimate.  Synchronises `stream`.
 */
slk_status slk_energy(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L,
                      const int32_t* labels, const float* z, const int32_t* modes_host, double lambda,
                      double sigma2, double delta, void* stream, slk_energy_out* out_host);

/*
 * Unary affinities and the initial assignment for fixed modes (Eq. (6a), Algorithm 1):
 * a_out[p, l] = k(x_p, x_{modes[l]}), z0_out = row softmax of a_out (device n x L float32;
 * either may be NULL).  Asynchronous.
 */
slk_status slk_unary(const float* x, int64_t n, int32_t d, int32_t L, const int32_t* modes_host,
                     double sigma2, slk_precision prec, void* stream, float* a_out, float* z0_out);

/*
 * One z-update from a given Z (Eqs. (6b), (8)) with a given unary matrix a (device n x L):
 * z_out = softmax(a + scale*lambda*(W + delta I) z_in); bound_host receives R(z_in) with
 * the factor scale*lambda/2 (host, may be NULL).  Synchronises `stream` if bound_host is
 * given.
 */
slk_status slk_inner_step(const slk_graph* g, int32_t L, const float* a, const float* z_in, double lambda,
                          double delta, int32_t pairwise_scale, void* stream, float* z_out,
                          double* bound_host);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the z-update of slk_inner_step without any
 * allocation, synchronisation or host output, so that it can also be captured into a HIP graph.
 *  g, L, a, z_in, lambda, delta, pairwise_scale : as in slk_inner_step (a, z_in: device n x L
 *                 float32, caller's layout and order).
 *  z_out        : device n x L float32 (may be NULL: bound only); must not alias z_in.
 *  bound_dev    : device, one double (may be NULL) receiving R(z_in) as in slk_inner_step.
 * The per-work-group bound partials and the pass state live in a 2 MiB array of device memory
 * that the library holds on every device it runs on until the process ends, so n is limited:
 * SLK_ERR_INVALID_ARG if n > slk_inner_step_noalloc_max_rows(L) (4,193,792 rows for 32 < L <= 256,
 * more for smaller L).  The array is shared by every call on one device and keeps the last
 * call's contents; the call resets what must start at zero itself.  Calls that overlap on one
 * device (different streams, or threads) race on the array: order them (one stream, or events).
 * The result equals slk_inner_step's up to the order of the floating-point sums (the rows are
 * walked by a different kernel).  The first call on a device looks up the array's address.
 */
slk_status slk_inner_step_noalloc(const slk_graph* g, int32_t L, const float* a, const float* z_in, double lambda,
                                  double delta, int32_t pairwise_scale, void* stream, float* z_out,
                                  double* bound_dev);

/* Largest n slk_inner_step_noalloc accepts for this L (0 if L is outside 1..256). */
int64_t slk_inner_step_noalloc_max_rows(int32_t L);

/*
 * Out-of-sample assignment (Section 1: the explicit assignment variables give a direct
 * out-of-sample extension).  Each query y takes the z-update of Eq. (8) once with the fit
 * held fixed:
 *   a_yl = k(y, m_l)  (Eq. (6a), Gaussian kernel with sigma2),
 *   b_y  = sum over the k nearest points q of y in x (binary kNN affinity, Section 4.2,
 *          ordered by (squared distance, index); the query is not excluded, it is not in x),
 *   z_y  = softmax(a_y + lambda b_y),  label_y = argmax_l (a_y + lambda b_y)_l (ties to the
 *          smaller l).
 *  x, n, d     : the fitted points (device, n x d float32).
 *  z, L        : their assignment Z (device, n x L float32, caller order), e.g. slk_fit's z_out.
 *  modes_host  : L mode indices into x (host).
 *  y, m        : queries (device, m x d float32).
 *  k           : neighbours per query, 1 <= k <= min(64, n).
 *  sigma2 > 0  : the kernel bandwidth (e.g. the graph's estimate from slk_graph_info).
 *  method, prec: kNN search and point precision, as in slk_build_knn.
 *  z_out       : m x L float32 (device); labels_out: m int32 (device, may be NULL);
 *  knn_idx_out : m x k int32 (device, may be NULL) receives the neighbours.
 *  Synchronises `stream`.
 */
slk_status slk_predict(const float* x, int64_t n, int32_t d, const float* z, int32_t L, const int32_t* modes_host,
                       const float* y, int64_t m, int32_t k, double lambda, double sigma2, slk_knn_method method,
                       slk_precision prec, void* stream, float* z_out, int32_t* labels_out, int32_t* knn_idx_out);

/*
 * SLK-MS mode update (Eq. (9)): with the assignment Z fixed, every mode is moved to the
 * weighted mean of the points, weights w_pl = z_pl k(x_p, m_l), and the step is repeated
 * until no mode moves by more than tol * sqrt(sigma2) in one step, or max_iter steps.
 * A cluster whose weights sum to zero keeps its mode.
 *  x, n, d     : points (device, n x d float32).
 *  z, L        : assignment (device, n x L float32), 1 <= L <= min(64, n).
 *  modes_in    : L x d float32 start vectors (device).
 *  sigma2 > 0  : the kernel bandwidth; prec: BF16 rounds the points (not the modes).
 *  modes_out   : L x d float32 (device; may equal modes_in).
 *  iters_host  : steps taken (host, may be NULL).  Sums are FP32 per 1,024-point block and
 *                FP64 across blocks.  Synchronises `stream`.
 */
slk_status slk_mean_shift(const float* x, int64_t n, int32_t d, const float* z, int32_t L, const float* modes_in,
                          double sigma2, double tol, int32_t max_iter, slk_precision prec, void* stream,
                          float* modes_out, int32_t* iters_host);

/*
 * SLK-MS (Algorithm 1 with the mean-shift mode update).  Each outer iteration runs the
 * z-update block of slk_assign with the unary term at the current mode vectors,
 * a_pl = k(x_p, m_l), then slk_mean_shift on the last z-update's Z (ms_tol, ms_max_iter).
 * The outer loop stops when no mode moved by more than ms_tol * sqrt(sigma2) over a whole
 * mode update (converged), or after params.max_outer.
 *  init_modes   : L x d float32 start vectors (device), e.g. L seeded points.
 *  z_out, labels_out : as in slk_assign, for the last outer iteration.
 *  modes_out    : L x d float32 (device), the modes after the last mean-shift.
 *  modes_used_out : L x d float32 (device, may be NULL), the modes the last z-updates used.
 *  ms_steps_host : total mean-shift steps (host, may be NULL).
 *  res_host     : as in slk_fit; energy at the last labels and modes_used_out.
 *  1 <= L <= 64.  Synchronises `stream`.
 */
slk_status slk_fit_ms(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L, const float* init_modes,
                      const slk_params* p, double ms_tol, int32_t ms_max_iter, void* stream, float* z_out,
                      int32_t* labels_out, float* modes_out, float* modes_used_out, int32_t* ms_steps_host,
                      slk_result* res_host);

/*
 * K-means++ seeding (Section 4.2 starts from K-means++ centres; the sampling rule is that of
 * Arthur and Vassilvitskii, 2007) and the nearest-seed assignment.
 *  u_host      : L uniforms in [0, 1) (host); the caller owns the random numbers.
 *  Centre 0 is the point floor(u_0 n).  Centre r >= 1 is the smallest p whose prefix sum of
 *  D^2 (in point order) exceeds u_r * sum D^2, where D^2(p) is the squared distance from x_p to
 *  the nearest centre chosen so far (FP64, coordinates summed in order, no FMA); if sum D^2 = 0
 *  it is floor(u_r n).  The prefix sums are formed per 256-point block and then across blocks;
 *  a choice can differ from that of a left-to-right sum only when the target lies within a few
 *  ulps of a prefix boundary.
 *  prec        : BF16 rounds the points before the distances.
 *  centres_out_host : L int32 (host).
 *  labels_out  : n int32 (device, may be NULL): index of the nearest centre (ties to the
 *                smaller index), the initial assignment.
 *  d2_out      : n double (device, may be NULL): D^2 after the last centre.
 *  Synchronises `stream`.
 */
slk_status slk_kmeanspp(const float* x, int64_t n, int32_t d, int32_t L, const double* u_host, slk_precision prec,
                        void* stream, int32_t* centres_out_host, int32_t* labels_out, double* d2_out);

/*
 * Exact modes by definition: Eq. (1), m_l = argmax over the points y of
 * P[y, l] = sum_p z_pl k(x_p, x_y) (the start modes of Section 4.2, from the initial
 * assignment), or with prev_host the proximal hard-max of Eq. (10), which adds k(x_y, x_prev_l).
 * Gaussian k with sigma2; ties to the smaller index.  Dense: 2 n^2 d + 2 n^2 L multiply-adds
 * on MFMA (centred points split into bf16 hi + lo; kernel values and Z split likewise; FP32
 * accumulation), so P carries a relative error of about 1e-5.
 *  z / labels  : exactly one: n x L float32 assignment (device) or n int32 hard labels (device;
 *                a label outside [0, L) adds nothing).
 *  prev_host   : L int32 (host, may be NULL): previous modes for Eq. (10).
 *  keep_host   : L int32 (host, may be NULL): the mode of a cluster with no weight (default
 *                prev_host; with neither, such a cluster is an SLK_ERR_INVALID_ARG).
 *  modes_out_host : L int32 (host); best_out_host : L float (host, may be NULL), the largest P.
 *  dens_out    : n x L float32 (device, may be NULL) receives P.
 *  1 <= L <= min(64, n).  Synchronises `stream`.
 */
slk_status slk_dense_modes(const float* x, int64_t n, int32_t d, int32_t L, const float* z, const int32_t* labels,
                           double sigma2, const int32_t* prev_host, const int32_t* keep_host, slk_precision prec,
                           void* stream, int32_t* modes_out_host, float* best_out_host, float* dens_out);

/*
 * Served and batched form (an extension; the paper fits one problem at a time).
 *
 * A job is one whole problem: its graph is built from its points (slk_build_knn with
 * job->knn) and SLK-BO (slk_fit) runs on it with job->params.  A server keeps up to
 * max_jobs jobs resident on the device and advances all of them together: each step packs
 * the work every resident job needs next (unary term, z-updates, final pass with labels and
 * modes, energy) into one launch per kernel, whatever the jobs' sizes, so many small problems
 * share the GPU.  Queued jobs are admitted whenever a slot is free and the job's estimated
 * device footprint fits the memory budget (continuous batching: jobs join and leave between
 * steps while the others keep running).  An admitted job's graph is built by one of
 * opts.builders worker threads, each on its own stream, while the resident jobs keep stepping;
 * the job joins the steps when its graph is ready.  Every job gets exactly the work-groups,
 * tiles and reduction order of its own slk_fit, so its outputs are bit-identical to running it
 * alone.
 *
 * slk_job: caller-owned descriptions and buffers, which must stay valid until the job is
 * reported done.
 *  x               : n x d float32 points (device).
 *  init_modes_host : L distinct int32 indices (host; copied by slk_server_submit).
 *  knn             : graph options (as slk_build_knn).
 *  params          : fit options (as slk_fit).
 *  z_out           : n x L float32 (device), labels_out: n int32 (device, may be NULL).
 *  modes_out_host, result_host, status_host : host outputs written when the job is done
 *                    (status SLK_OK, or the error that stopped this job alone).
 * Limits of the served form: 1 <= L <= 64 (jobs with larger L are rejected with
 * SLK_ERR_UNSUPPORTED; use slk_fit).
 */
typedef struct {
  const float* x;
  int64_t n;
  int32_t d;
  int32_t L;
  const int32_t* init_modes_host;
  slk_knn_opts knn;
  slk_params params;
  float* z_out;
  int32_t* labels_out;
  int32_t* modes_out_host;
  slk_result* result_host;
  slk_status* status_host;
} slk_job;

typedef struct {
  int32_t max_jobs;         /* resident jobs (slots); 1 <= max_jobs <= 1024                    */
  int32_t passes_per_step;  /* z-updates queued per step for jobs in their inner loop (>= 1)    */
  int64_t memory_budget;    /* bytes of device memory the resident jobs may use (0 = 80% of
                               the free memory when the server is created)                     */
  int32_t builders;         /* worker threads building admitted jobs' graphs, each on its own
                               stream, while the resident jobs step; 1 <= builders <= 8        */
  int32_t graph_replay;     /* 1: a step's launch sequence is captured into a HIP graph the
                               second time its shape (kernels, grids, argument layout) occurs,
                               and replayed whenever that shape recurs; 0: plain launches.
                               The same kernels run on the same arguments either way.  Takes
                               effect for a server created on a non-null stream (the null
                               stream cannot be captured).                                     */
} slk_server_opts;

typedef struct slk_server slk_server;

/* Fill *o with defaults: max_jobs 64, passes_per_step 4, memory_budget 0, builders 3,
   graph_replay 1. */
slk_status slk_server_opts_default(slk_server_opts* o);

/* Create a server that runs on `stream` (device = the current device).  Release with
   slk_server_destroy (which drops unfinished jobs). */
slk_status slk_server_create(const slk_server_opts* opts, void* stream, slk_server** out);

/* Queue a job; *ticket_host receives its id (0, 1, 2, ... in submission order).  Checks the
   job's arguments at once (n >= 2, d >= 1, 1 <= L <= min(64, n), modes distinct and in range,
   parameters and kNN options valid). */
slk_status slk_server_submit(slk_server* sv, const slk_job* job, int64_t* ticket_host);

/* Admit what fits (queued jobs go to the graph builders), take in the jobs whose graphs are
   ready, then run one step for every resident job and synchronise the server's stream.  With no
   resident job and graphs still being built, waits for the first of them.  done_host (may be
   NULL) receives up to `cap` tickets of jobs finished in this or an earlier step and not yet
   reported; *n_done_host their number.  *n_active_host and *n_queued_host (may be NULL) receive
   the resident and the waiting job counts (queued or in a graph build) after the step. */
slk_status slk_server_step(slk_server* sv, int64_t* done_host, int32_t cap, int32_t* n_done_host,
                           int32_t* n_active_host, int32_t* n_queued_host);

typedef struct {
  int64_t steps;            /* slk_server_step calls that ran resident jobs                       */
  int64_t graph_launches;   /* steps replayed from a captured HIP graph                           */
  int64_t graph_captures;   /* step shapes captured                                               */
  int64_t grouped_builds;   /* shared launches of the exact kNN search for several jobs           */
} slk_server_stats_t;

/* Counters of the server's work so far (host). */
slk_status slk_server_stats(const slk_server* sv, slk_server_stats_t* out_host);

void slk_server_destroy(slk_server* sv);

/* Fit every job in jobs[0 .. n_jobs-1] with a server (opts may be NULL: defaults) and return
   when all are done.  Per-job failures are reported in their status_host; the call itself
   fails only for invalid arguments or a device error. */
slk_status slk_fit_batched(const slk_job* jobs, int32_t n_jobs, const slk_server_opts* opts, void* stream);

/*
 * Per-kernel timing for measurement: with timing on, every launch of the timed kernels
 * ("unary_kernel", "iter_kernel", "final_kernel", "mode_reduce_kernel", "energy_kernel" of
 * slk_assign / slk_fit; "cand_kernel", "rerank_kernel" of the MFMA kNN; "kpp_dist_kernel",
 * "kpp_select_kernel", "dmode_kernel", "ms_partial_kernel" of the extensions) is bracketed by
 * two HIP events recorded on the call's stream, and the elapsed times are accumulated per
 * kernel name.  slk_timing_enable(on) clears the totals and switches timing on (1) or off (0);
 * slk_timing_read first waits for the launches still pending, then returns the number of timed
 * launches and their total milliseconds for one kernel name (0 and 0.0 if none).  Process-wide
 * state; timing adds one event pair per launch and should stay off in production.
 */
slk_status slk_timing_enable(int32_t on);
slk_status slk_timing_read(const char* kernel, int64_t* launches_host, double* total_ms_host);

/* Returns the work memory the library keeps on the current device (the blocks of the
   synchronising calls and the pool's freed memory) to the system.  Memory of calls still in
   progress on any thread or stream stays allocated; later calls allocate again as they need.
   For callers that must bound the device memory the library holds between calls.
   SLK_ERR_DEVICE if the pool cannot be created or trimmed. */
slk_status slk_pool_trim(void);

/*
 * Tile shapes.  The z-update and final pass walk each work-group's rows in tiles of
 * wave_steps row batches per wave; the exact kNN puts knn_exact_width queries in a work-group.
 * They come from a table the project's autotuner (tune.py) measured on the GPU, keyed by the row
 * count and the lane-group class of L, and every call - single fits, assignments, the served form
 * - takes them from there, so a job's results are the same wherever it runs.  Tile shapes change
 * no result except the order of the relaxed bound's FP64 partial sums.  knn_long_scan reports the
 * form of the MFMA candidate search over n keys (the candidate lists are the same either way).
 */
typedef struct {
  int32_t wave_steps;       /* row batches per wave in a z-update tile (L <= 64; 4 above)       */
  int32_t knn_exact_width;  /* queries per work-group of the exact kNN over n rows              */
  int32_t knn_exact;        /* 1 if the AUTO kNN method takes the exact search for (n, d)        */
  int32_t knn_long_scan;    /* 1 if the MFMA candidate search over n keys tests each key tile
                               against all of a wave's rows before merging (n >= 393,216)         */
} slk_tune_params;

/* The tile shapes a problem of n points in d dimensions with L clusters gets (host output). */
slk_status slk_tune_lookup(int64_t n, int32_t d, int32_t L, slk_tune_params* out_host);

/* For the autotuner's measurements only: force the z-update's wave_steps (1, 2, 4 or 8) for every
   later call in the process, or go back to the table (0).  Not for use while calls are running. */
slk_status slk_tune_override(int32_t wave_steps);

/* Where the table came from (the autotuner's run: device and date), for reports. */
const char* slk_tune_source(void);

/* Text for the last non-OK status returned on this thread. */
const char* slk_last_error(void);

/* Library version string. */
const char* slk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SLK_H_ */
