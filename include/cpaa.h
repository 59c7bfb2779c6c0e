/*
 * cpaa.h - C ABI of the MI355X (gfx950) implementation of the Chebyshev
 * Polynomial Approximation Algorithm (CPAA) for PageRank on undirected graphs
 * (Zhang, Tang, Yao, Zhang, "A Parallel PageRank Algorithm For Undirected
 * Graph", arXiv 2112.01743).
 *
 * What is computed (Sec. 2.1, Sec. 3 eq. 3.1, Sec. 4.1 Alg. 1):
 *   P = A D^{-1} is the random-walk matrix of an undirected graph (A the 0/1
 *   symmetric adjacency pattern, D the degrees), c in (0,1) the damping
 *   factor, p a personalization vector.  PageRank is
 *       pi = (1 - c) (I - cP)^{-1} p.
 *   CPAA approximates (I - cP)^{-1} b, b = (1-c) p, by the truncated Chebyshev
 *   series of f(x) = 1/(1 - cx):
 *       x_M = (c_0/2) b + sum_{k=1..M} c_k T_k(P) b,    c_k = 2 beta^k / sqrt(1-c^2),
 *   with T_{k+1}(P)b = 2 P T_k(P)b - T_{k-1}(P)b (Sec. 2.2 property (3)) and
 *   beta = (1 - sqrt(1-c^2))/c (eq. 4.1).
 *
 * Precision: the recurrence runs in FP32; the weighted accumulation of the
 * series, the residual r = b - (I - cP)x and the returned vector are FP64.
 * Every solve ends with an FP64 residual; ||r||_1/(1-c) bounds ||x - pi||_1
 * (||(I-cP)^{-1}||_1 = 1/(1-c) for column-stochastic P).  If that bound is
 * above the requested tolerance the library runs correction series on r
 * (x += x_M(r)), at most cpaa_opts.max_refine times.
 *
 * Conventions for every entry point:
 *   - The caller owns every buffer it passes; the library never frees or
 *     keeps caller pointers beyond the call.  A plan owns device copies of the
 *     graph and its own workspace.
 *   - Functions return a cpaa_status and never throw or abort across the ABI.
 *     On an error other than CPAA_ENOCONV the outputs are left untouched and
 *     cpaa_last_error() describes the failure (thread-local string).
 *   - "device pointer" means memory from hipMalloc (or a torch HIP tensor) on
 *     the device that was current when the plan was made.
 *   - Work is enqueued on the HIP stream passed as `stream` (NULL = default
 *     stream); solve calls return after the results are in `x`.
 *   - Calls that share one plan must not overlap (the plan's workspace is
 *     reused); different plans are independent.
 */
#ifndef CPAA_H
#define CPAA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPAA_API __attribute__((visibility("default")))

typedef struct cpaa_plan_s* cpaa_plan_t;

typedef enum {
  CPAA_OK = 0,
  CPAA_EINVAL = 1,      /* bad argument: null pointer, c not in (0,1), tol <= 0, bad sizes,
                           non-finite or negative p, p not summing to 1 */
  CPAA_ENOTSYM = 2,     /* adjacency pattern is not symmetric (graph not undirected) */
  CPAA_EISOLATED = 3,   /* a vertex of degree 0: P = A D^{-1} is undefined there (Sec. 2.1) */
  CPAA_ESELFLOOP = 4,   /* a self loop */
  CPAA_EPATTERN = 5,    /* row_ptr not monotone, column out of range, unsorted or duplicate */
  CPAA_ENOMEM = 6,      /* device or host allocation failed */
  CPAA_EDEVICE = 7,     /* HIP runtime error */
  CPAA_ENOCONV = 8      /* tolerance not certified within the term / refinement caps;
                           the best-effort x and its report are still written */
} cpaa_status;

/* Graph input: the symmetric 0/1 pattern in CSR form, int32 indices.
 * Each undirected edge {u,v} is stored twice (u->v and v->u); columns sorted
 * within each row; no self loops, no duplicates, no isolated vertices.
 * Only the pattern is read: Alg. 1 uses N(u) and deg(v) (Sec. 4.1), no
 * per-edge values. */
typedef struct {
  int32_t n;                 /* vertices */
  int64_t nnz;               /* stored entries = 2|E| (the paper's m), < 2^31 */
  const int32_t* row_ptr;    /* [n+1], row_ptr[0] = 0, row_ptr[n] = nnz */
  const int32_t* col_idx;    /* [nnz] */
  int32_t num_graphs;        /* 0 or 1: one graph.  > 1: block-diagonal batch of independent
                                graphs, solved with cpaa_solve_graphs */
  const int32_t* graph_ptr;  /* [num_graphs+1] first vertex of each graph (num_graphs > 1) */
  int32_t on_device;         /* 1: row_ptr/col_idx/graph_ptr/values are device pointers, 0: host */
  const double* values;      /* [nnz] or NULL.  Optional entries of P = A D^-1 (Sec. 2.1): the
                                entry in column v must be 1/deg(v) (1/out-degree of v in a
                                directed plan) to within 4 ulps, else CPAA_EINVAL.  Checked,
                                then not used (only the pattern is read). */
} cpaa_csr;

typedef struct {
  int32_t k_max;          /* cap on terms of one series; 0 = from the a-priori bound (<= 512) */
  int32_t max_refine;     /* FP64-residual correction series allowed (default 2) */
  int32_t normalize;      /* 1: divide each result by its sum (Alg. 1's last step);
                             plain solves only, changes what tol certifies (see cpaa_solve) */
  int32_t nnz_per_thread; /* 0 auto; 4, 8, 16 or 32: stored entries per thread of a single-vector
                             work item (a workgroup of 256 threads takes 256*this entries and the
                             rows they cover, so rows per wavefront = this*64/degree) */
  int32_t tile_w;         /* 0 auto; 8, 16, 32 or 64: right-hand sides per tile in batched solves */
  int32_t validate;       /* 1 (default): check the pattern (symmetry, loops, order) on the host */
  int32_t io_device;      /* 1 (default): p / x0 / x of solve calls are device pointers; 0: host */
  int32_t time_kernels;   /* device time of the term kernels with HIP events (report.ms_terms):
                             1 one pair of events around every term launch, 2 one pair around
                             each series of back-to-back term launches (the convergence checks
                             between them included).  An event between two launches leaves the
                             GPU idle for about 10 us, so 1 slows a solve down; 2 does not. */
  int32_t xcd_remap;      /* -1 auto (off for single-vector kernels, on for tiled kernels),
                             0/1: map workgroups to contiguous row ranges per XCD */
  int32_t autotune;       /* 1: the first call of each solve path times its candidate launch
                             shapes on its own input and keeps the fastest for the plan:
                             cpaa_solve (plain solve): work maps of 8/16/32 entries per thread
                             (when nnz_per_thread = 0) in row order, or the launch shape of the
                             column-sliced gather pass (when slice_shape = 0);
                             cpaa_solve_batched: tile_w 16/32/64
                             (when tile_w = 0); cpaa_solve_graphs: 256/512/1024 threads per
                             graph */
  int32_t column_slices;  /* single-vector path: 0 auto, 1 off, 8 on.  On: vertices are relabelled
                             by degree rank dealt round-robin into 8 contiguous slices (equal
                             size and near-equal degree sum); each term's SpMV then runs per
                             column slice, slice s on the workgroups the hardware places on XCD
                             s, so every XCD gathers from one eighth of the vector, which stays
                             in its L2, and a combine pass adds the 8 partial row sums and
                             applies the term update.  Auto: on for one graph with n >= 3 * 2^18
                             and max degree >= 16 x average degree (for a directed plan also
                             when its entries span more than 2^14 labels on average).  Needs
                             one graph and n < 8 (2^21 - 16) (else CPAA_EINVAL).  Inputs and
                             outputs keep the caller's labels. */
  int32_t locality_order; /* single-vector path without column slices: 0 auto, 1 off (caller's
                             labels), 2 reverse Cuthill-McKee.  RCM relabels the vertices by a
                             breadth-first order from a pseudo-peripheral vertex, so that on
                             mesh-like graphs the columns of neighbouring rows are close and a
                             term's gathers stay in L2.  Auto: for one graph with n >= 2^18
                             whose stored entries span more than 2^14 labels on average, if RCM
                             shortens that mean span at least 8x.  Inputs and outputs keep the
                             caller's labels. */
  int32_t spectral_interval; /* 0 (default): the Chebyshev expansion on [-1, 1] (Alg. 1).
                             1: estimate the smallest eigenvalue lambda_min of P at plan time
                             (80 Lanczos steps on D^{-1/2} A D^{-1/2} on the host) and expand on
                             [a, 1], a = lambda_min - 0.02 (Sec. 2.2's general interval; kept at
                             -1 when a < -0.95, e.g. for graphs with a bipartite component):
                             fewer terms when the spectrum stays away from -1.  Results are
                             certified as always; a wrong a only slows convergence.  Single-graph
                             plans only (else CPAA_EINVAL); the power method ignores it. */
  int32_t directed;       /* 1: a directed graph (Sec. 2.1: a_uv = 1 iff v -> u): row u lists the
                             vertices v with an edge v -> u, columns sorted, no duplicates or
                             self loops; symmetry is not required and rows may be empty.  The
                             out-degree of v is the number of rows listing v; a vertex without
                             out-edges is dangling, and P' = P + p d^T sends its mass along p
                             (Sec. 2.1).  CPAA's expansion needs the real spectrum of an
                             undirected graph (Sec. 3), so every solve of such a plan runs the
                             power method: cpaa_solve falls back to it (report.method = 1), and
                             the batched calls solve their columns one after another through
                             the single-vector path.  No warm start (x0 / X0 must be NULL, else
                             CPAA_EINVAL).  Needs one graph; RCM and the spectral interval are
                             not used (CPAA_EINVAL when asked for); column slices are.
                             2: detect.  The plan is directed if the pattern is not symmetric or
                             has an empty row (a vertex without edges, dangling), else
                             undirected; the other pattern rules are checked as for 1.
                             cpaa_plan_info_get reports which. */
  int32_t slice_shape;    /* column-sliced term of an undirected plan: launch shape of its gather
                             pass, 0 auto (shape 1; with autotune the first cpaa_solve times the
                             shapes 1-4 and keeps the fastest), 1-4 a fixed shape, given as
                             wavefronts per workgroup / vertices of the slice kept in LDS:
                             1 = 16 / 16,384, 2 = 8 / 8,192 (two workgroups per CU),
                             3 = 4 / 2,048, 4 = 16 / 22,528; 5 = the per-item layout (dense
                             partial sums, the layout of directed plans).  Shapes 1-4 give
                             identical results; only their speed differs. */
  int32_t fp64_recurrence; /* 1: debug mode, the Chebyshev (and power-method) recurrence in FP64
                             instead of FP32 (the accumulation, residual and certificate are FP64
                             always): results then follow the FP64 oracle's x_M to rounding.
                             Row order only (no column slices; CPAA_EINVAL with column_slices = 8),
                             one undirected graph; batched calls solve their columns one after
                             another through the single-vector path. */
  int32_t deterministic;  /* 1: bitwise-reproducible results: every sum is formed in a fixed order
                             (partial row sums by a fixed-order scan, per-block partials of every
                             reduction added in block order, no floating-point atomics), so two
                             solves of the same input on the same device return identical bits.
                             Uses the column-sliced term (forced on, any n); one undirected graph;
                             batched calls solve their columns one after another. */
  int32_t drop_isolated;  /* 1: accept vertices without edges (undirected plans).  P = A D^-1 has a
                             zero column there (Sec. 2.1 needs d_v > 0), so (I - cP) x = (1-c) p
                             gives x_v = (1-c) p_v, and no other vertex depends on v: the plan
                             solves the graph without them (relabelled internally) and writes
                             x_v = (1-c) p_v (scaled like the rest under normalize) for each
                             dropped v.  0 (default): such a vertex is CPAA_EISOLATED. */
  int32_t rows_per_wave;  /* column-sliced term with compact partials (undirected plans): most
                             rows one wavefront's work item may hold, 1-1024; 0 (default) =
                             1024.  An item also holds at most 2,048 stored entries, so the cap
                             only binds where rows have few entries in a slice; smaller caps
                             give more, shorter items.  The row-order layout is sized by
                             nnz_per_thread instead.  Results depend on it only through the
                             summation order of a row's entries. */
} cpaa_opts;

/* Per-solve report (one per right-hand side in batched calls, one per graph in
 * cpaa_solve_graphs). */
typedef struct {
  int32_t terms;          /* Chebyshev terms M of the main series */
  int32_t refine_terms;   /* terms summed over all correction series */
  int32_t refinements;    /* correction series run */
  int32_t certified;      /* 1 if cert_bound <= tol */
  int32_t fallback_used;  /* warm start rejected and a plain solve done instead */
  int32_t method;         /* 0 CPAA (Chebyshev series), 1 the power method (cpaa_solve_power*,
                             and every solve of a directed plan) */
  double cert_bound;      /* ||r||_1/(1-c) in FP64: upper bound on ||x - pi||_1 (before normalize) */
  double resid_l1;        /* ||r||_1, r = b - (I - cP)x */
  double resid_max;       /* ||r||_inf */
  double mass;            /* sum_i x_i */
  double series_cert;     /* in-loop bound of the last series (from its last two terms) */
  double ms_total;        /* device time of the whole call (events on `stream`) */
  double ms_terms;        /* device time of the term launches (time_kernels = 1 or 2), whole call */
  int64_t term_launches;  /* term launches that did work within ms_terms */
  int64_t edges;          /* nnz x terms (main + correction) processed for this right-hand side */
} cpaa_report;

/* Plan facts, for diagnostics and benchmarks. */
typedef struct {
  int32_t n;
  int64_t nnz;
  int32_t num_graphs;
  int32_t reordered;        /* single-vector labelling: 0 the caller's, 1 column slices (degree
                               rank), 2 reverse Cuthill-McKee */
  int32_t max_degree;
  int32_t split_rows;       /* rows split across workgroups */
  int32_t nnz_per_thread;   /* single-vector work item size / 256 */
  int32_t work_items;       /* single-vector workgroups per term */
  int32_t tile_w;           /* batched tile width in use */
  int32_t k_cap_global;     /* a-priori term cap for uniform p at tol 1e-6 */
  double c;
  double beta;              /* decay ratio of the coefficients in use (of c' on [a, 1]) */
  double vol;               /* sum of degrees */
  int32_t column_slices;    /* single-vector term: 1 (row order) or 8 (column-sliced) */
  double spectrum_lo;       /* a of the expansion interval [a, 1] (-1: the paper's) */
  int32_t directed;         /* 1 for a directed plan (opts.directed = 1, or 2 and detected) */
  int32_t slice_shape;      /* launch shape of the column-sliced gather pass in use (1-4; 5 the
                               per-item layout), 0 when the plan has no such pass */
  int64_t slice_partials;   /* partial row sums per term of the column-sliced term: rows with an
                               entry in a slice, summed over the 8 slices */
} cpaa_plan_info;

/* Fill *o with defaults.  Never fails. */
CPAA_API void cpaa_default_opts(cpaa_opts* o);

/* Build a plan for graph g and damping c (Sec. 2.1).  Validates the pattern
 * (if opts->validate), computes degrees, the work-item maps, the coefficient
 * table c_k (Prop. 1: c_k = c_0 beta^k), and uploads the pattern to the
 * current device.  With column slices (opts->column_slices) the plan also
 * holds a relabelled copy of the pattern and the per-slice packed entries:
 * about three times the pattern's 4 (n + 1 + nnz) bytes in device memory, plus
 * 32 n bytes of partial sums once a solve runs.  For a block-diagonal batch
 * (num_graphs > 1) it packs each graph's entries for cpaa_solve_graphs.
 * opts may be NULL (defaults).
 * Errors: CPAA_EINVAL, CPAA_ENOTSYM, CPAA_EISOLATED, CPAA_ESELFLOOP,
 * CPAA_EPATTERN, CPAA_ENOMEM, CPAA_EDEVICE.  On success *out owns the plan. */
CPAA_API cpaa_status cpaa_plan(const cpaa_csr* g, double c, const cpaa_opts* opts, cpaa_plan_t* out);

/* Release every device and host resource of the plan.  NULL is ignored. */
CPAA_API void cpaa_plan_destroy(cpaa_plan_t plan);

/* Copy the plan's facts into *info. */
CPAA_API cpaa_status cpaa_plan_info_get(cpaa_plan_t plan, cpaa_plan_info* info);

/* One solve (single-graph plan).
 *   p   : [n] FP64 personalization, p >= 0, sum p = 1 (Sec. 2.1: an
 *         n-dimensional probability distribution).
 *   tol : target for ||x - pi||_1, certified by the FP64 residual (> 0).
 *   x0  : NULL for a plain solve (b = (1-c)p).  Otherwise a starting guess
 *         [n]: the library forms r0 = (1-c)p - (I-cP)x0 in FP64 and runs CPAA
 *         on b = r0 (x = x0 + x_M(r0)); if x0 is not finite or not better than
 *         zero (||r0||_1 >= (1-c)||p||_1) it falls back to the plain solve and
 *         sets report.fallback_used.
 *   x   : [n] FP64 output, in the caller's vertex order.
 *   rep : may be NULL.
 * Pointers are device pointers if opts.io_device = 1, host pointers otherwise.
 * With opts.normalize = 1 the result is divided by its sum after
 * certification; the bound in the report refers to the unnormalized x.
 * On a directed plan (opts.directed) the call runs the power method instead
 * (as cpaa_solve_power; x0 must be NULL) and sets report.method = 1.
 * Returns CPAA_OK when certified, CPAA_ENOCONV when not (x still written). */
CPAA_API cpaa_status cpaa_solve(cpaa_plan_t plan, const double* p, double tol, const double* x0,
                       double* x, cpaa_report* rep, void* stream);

/* cpaa_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve (Chebyshev series, FP64 residual, corrections, warm start), with
 * its workspace in a static device array of the library (64 MiB per device,
 * held until the process ends) instead of buffers the plan allocates, and no
 * timing events.  Calls on one device share that array and the library's host
 * mirror of the statistics, so calls that overlap in time on a device race
 * (run them one after another).  Needs an undirected single-graph plan made on
 * the current device with io_device = 1 (p, x0, x device pointers), and a
 * workspace that fits the array (about 40-60 bytes per vertex plus 0.3 MB:
 * n up to about 1M); otherwise CPAA_EINVAL and nothing is written.  The FP64
 * residual of a column-sliced plan runs as in cpaa_solve (per column slice)
 * when its partial sums fit the array too, else in row order (the same value
 * up to rounding).  It calls no hipMalloc, hipFree or other allocating
 * routine; the plan's own device memory is made by cpaa_plan. */
CPAA_API cpaa_status cpaa_solve_noalloc(cpaa_plan_t plan, const double* p, double tol,
                                        const double* x0, double* x, cpaa_report* rep,
                                        void* stream);

/* B solves at once: column j of P is P[j*ldp + i], i < n, likewise X0 (may be
 * NULL) and X.  The right-hand sides are processed in tiles of opts.tile_w
 * columns by one SpMM kernel per term; each tile stops when all its columns
 * are certified (per-column in-loop certificate), and each column gets its own
 * FP64 residual and report.  On a directed plan the columns are solved one
 * after another by the single-vector power method (X0 must be NULL); plans
 * with fp64_recurrence, deterministic or dropped vertices also solve their
 * columns one after another through cpaa_solve.  A column that fails
 * validation stops the call with its error, and the columns before it are
 * already written.  reps: [B] or NULL.  ldp, ldx0, ldx >= n.
 * A block-diagonal plan (num_graphs > 1) takes B = 1: the one column holds
 * every graph's personalization at that graph's vertices (each part a
 * distribution), X0 must be NULL, and reps receives num_graphs reports; the
 * call is cpaa_solve_graphs.  Other rules as cpaa_solve. */
CPAA_API cpaa_status cpaa_solve_batched(cpaa_plan_t plan, int32_t B, const double* P, int64_t ldp,
                               double tol, const double* X0, int64_t ldx0, double* X,
                               int64_t ldx, cpaa_report* reps, void* stream);

/* The power method on the same plan and kernels, the baseline the paper
 * compares CPAA with (Sec. 5, Table 3).  PageRank is the fixed point of
 * pi = P''pi (eq. 2.1); for an undirected graph this is the iteration
 *     x_{t+1} = c P x_t + (1-c) p,    x_0 = p,
 * whose iterates stay distributions and whose error shrinks by c per step.
 * The library sums it as x_0 plus its increments x_{t+1} - x_t = (cP)^t
 * (x_1 - x_0): FP32 increments, FP64 sum, stopped when the FP64 norm of the
 * next increment (the residual of the current iterate) certifies
 * ||x_t - pi||_1 <= tol/2, then the same FP64 residual check and corrections
 * as cpaa_solve (a correction runs the iteration on b = r from x_0 = r/(1-c)).
 * report.terms counts power-method steps (one SpMV each).  With
 * opts.k_max = t, opts.max_refine = 0 and a tolerance that cannot be met the
 * output is the t-th iterate x_t itself (and CPAA_ENOCONV is returned).
 * Arguments, validation, x0 handling, ownership and errors as cpaa_solve. */
CPAA_API cpaa_status cpaa_solve_power(cpaa_plan_t plan, const double* p, double tol,
                                      const double* x0, double* x, cpaa_report* rep,
                                      void* stream);

/* B power-method solves at once, as cpaa_solve_batched (tiles of columns, one
 * SpMM kernel per step, per-column certificates and reports). */
CPAA_API cpaa_status cpaa_solve_power_batched(cpaa_plan_t plan, int32_t B, const double* P,
                                              int64_t ldp, double tol, const double* X0,
                                              int64_t ldx0, double* X, int64_t ldx,
                                              cpaa_report* reps, void* stream);

/* Block-diagonal plan (num_graphs > 1): solve every graph for its own
 * personalization in one persistent kernel launch (one workgroup per graph at
 * a time, vectors resident in LDS, terms per graph chosen by its own in-loop
 * certificate), followed by the FP64 residual of every graph.
 *   p   : [n] concatenated personalizations; the block of graph g sums to 1.
 *   x   : [n] concatenated results.
 *   reps: [num_graphs] or NULL.
 * Returns CPAA_OK if every graph is certified, CPAA_ENOCONV otherwise. */
CPAA_API cpaa_status cpaa_solve_graphs(cpaa_plan_t plan, const double* p, double tol, double* x,
                              cpaa_report* reps, void* stream);

/* ---- Learned warm start --------------------------------------------------
 * A message-passing network of `layers` layers of width 64 over the plan's
 * graph predicts a personalized PageRank vector x0 from each vertex's log
 * degree and a one-hot source; pass its output as x0 / X0 to cpaa_solve /
 * cpaa_solve_batched, which run CPAA on the residual and fall back to the
 * plain solve when x0 is rejected.  Per layer l: M = A D^{-1} H (the paper's
 * P, Sec. 2.1), Z = H W_self + M W_nbr + b, H' = relu(Z); head:
 * x0 = softmax over the vertices of H w_out + b_out (clamped to +-80).  bf16 weights and
 * activations, FP32 accumulation (MFMA for the width-64 layers), FP32
 * gradients, Adam on FP32 master weights.
 * Parameter packing (FP32, host arrays): for l = 0..layers-1: W_self^l
 * (fan_in x 64 row-major, fan_in = 2 for l = 0 else 64), W_nbr^l (same), b^l
 * (64); then w_out (64), b_out (1).  cpaa_model_num_params gives the count.
 * The model keeps a pointer to the plan, which must outlive it. */
typedef struct cpaa_model_s* cpaa_model_t;

/* Create a model on a single-graph plan with the given initial parameters
 * (host).  hidden must be 64, layers 1..4.  Errors: CPAA_EINVAL, CPAA_ENOMEM,
 * CPAA_EDEVICE. */
CPAA_API cpaa_status cpaa_model_create(cpaa_plan_t plan, int32_t layers, int32_t hidden,
                                       const float* params, cpaa_model_t* out);
CPAA_API void cpaa_model_destroy(cpaa_model_t model);
CPAA_API int32_t cpaa_model_num_params(cpaa_model_t model);

/* Copy out / restore the FP32 master parameters, Adam moments and step count
 * (host arrays of cpaa_model_num_params floats; NULL skips an array).  Used
 * for checkpoints and resuming training. */
CPAA_API cpaa_status cpaa_model_get_state(cpaa_model_t model, float* params, float* adam_m,
                                          float* adam_v, int64_t* step);
CPAA_API cpaa_status cpaa_model_set_state(cpaa_model_t model, const float* params,
                                          const float* adam_m, const float* adam_v,
                                          int64_t step);

/* x0 for B sources (host int32 array): column j written to X0[j*ldx + i]
 * (device FP64).  Synchronous on `stream`. */
CPAA_API cpaa_status cpaa_model_predict(cpaa_model_t model, int32_t B, const int32_t* sources,
                                        double* X0, int64_t ldx, void* stream);

/* One training step on B sources against targets T (device FP64, column j at
 * T[j*ldt]; normally plain CPAA results): forward, cross-entropy loss
 * -sum_u T_u log x0_u, backward, gradient averaged over the sources, then Adam
 * with learning rate lr if lr > 0.  grads_out (host, may be NULL) receives the
 * averaged gradient (before the update); loss_out (host, may be NULL) the
 * mean L1 distance sum_u |x0_u - T_u| of the step's guesses. */
CPAA_API cpaa_status cpaa_model_train_step(cpaa_model_t model, int32_t B, const int32_t* sources,
                                           const double* T, int64_t ldt, float lr,
                                           float* grads_out, double* loss_out, void* stream);

/* Thread-local description of the last error ("" if none). */
CPAA_API const char* cpaa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CPAA_H */
