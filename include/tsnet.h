/*
 * tsnet.h -- C ABI of the MI355X (gfx950) L-tsNET gradient library.
 *
 * The library computes, on one GPU, the per-iteration gradient of the tsNET
 * cost (Eq. 1 of Meidiana, Hong and Ma, "BH-tsNET, FIt-tsNET, L-tsNET: Fast
 * tsNET Algorithms for Large Graph Drawing") the way L-tsNET does it
 * (Algorithm 3, Sec. 3.3): a sparse attractive KL term over the partial-BFS
 * affinities P, FFT-accelerated interpolation for the KL repulsion with its
 * normaliser Z, the same interpolation for the entropy sums of Eq. (8), the
 * compression term, and the vertex move.
 *
 * Conventions shared by every call:
 *  - Return value: TSNET_OK (0) or a negative TSNET_E* code. No C++
 *    exception crosses this boundary. tsnet_last_error() returns a message
 *    for the calling thread's most recent failure.
 *  - Pointers are DEVICE pointers unless the name or comment says host.
 *    Device buffers passed in are owned by the caller and must stay alive
 *    until the enqueued work that uses them has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls validate their arguments on the host, then enqueue asynchronously
 *    on `stream`, except where a call is marked "synchronous".
 *  - Layout: X, G, F_* and update/gains are row-major [n][2] float (x, y).
 *    Vertex ids are global across a batch of graphs; graph g owns the
 *    vertices [graph_offsets[g], graph_offsets[g+1]) and is an independent
 *    layout problem with its own n, P normalisation, grid and Z.
 *  - A context must not be used from two threads at once. Calls on one
 *    context and one stream are ordered; the library uses no other stream.
 */
#ifndef TSNET_H
#define TSNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSNET_OK       0
#define TSNET_EINVAL  (-1)   /* bad argument, bad CSR, unsupported size      */
#define TSNET_EHIP    (-2)   /* HIP runtime error                              */
#define TSNET_ENOMEM  (-3)   /* device allocation failed                       */
#define TSNET_EGRID   (-4)   /* non-finite layout (NaN/Inf) seen by the grid   */

/* tie_mode of tsnet_build_P */
#define TSNET_TIE_HASH 0     /* key = SplitMix64 hash of (seed, source, target) */
#define TSNET_TIE_ID   1     /* key = target id                                 */

/* attract_layout of tsnet_params: how the attractive sum over P is laid out */
#define TSNET_ATTRACT_AUTO  0  /* tiled from 262144 vertices on, else rows        */
#define TSNET_ATTRACT_ROWS  1  /* one wave per CSR row, x_j gathered from HBM     */
#define TSNET_ATTRACT_TILED 2  /* row tiles x column windows, x_j read from LDS   */

/* How the repulsion (with Z) and the entropy sums are computed (tsnet_params). */
#define TSNET_TERMS_INTERP   0  /* FFT-accelerated interpolation (L-tsNET, Sec. 3.3) */
#define TSNET_TERMS_QUADTREE 1  /* Barnes-Hut quadtree (BH-tsNET / FIt-tsNET, Eq. 7) */

/* bits of the device status word (tsnet_status) */
#define TSNET_STATUS_NONFINITE   0x1u  /* NaN/Inf in X at some grid set-up          */
#define TSNET_STATUS_GRID_CAPPED 0x2u  /* span / interval_width > max_intervals      */
#define TSNET_STATUS_ROW_LOW     0x4u  /* some row could not reach u from below      */
#define TSNET_STATUS_ROW_HIGH    0x8u  /* some row could not reach u from above      */
#define TSNET_STATUS_ROW_EMPTY   0x10u /* some vertex has no neighbour               */
#define TSNET_STATUS_WORKSPACE   0x20u /* a batch's grids were planned down to fit the
                                          evaluation workspace (with GRID_CAPPED)     */

typedef struct tsnet_ctx_s* tsnet_ctx;   /* per-device state: twiddles, status, timers */
typedef struct tsnet_P_s*   tsnet_P;     /* one problem: graph batch, P, workspace      */

/*
 * Cost weights and interpolation settings.
 *  lambda_kl, lambda_c, lambda_r: the multipliers of Eq. (1) (Sec. 2.1).
 *  eps_r: the entropy regulariser epsilon (1/20, Sec. 3.3).
 *  interval_width: target box side h of the interpolation grid; the box count
 *    per axis is ceil(span / h) clamped to [min_intervals, max_intervals] and
 *    rounded up to a power of two (the paper leaves I and P open, Sec. 2.3).
 *    span is the larger side of the region the grid covers: the bounding box
 *    of the graph's layout, or its core when far points are set apart.
 *  far_trim: t of the far-point rule (Sec. 2.3 leaves the covered region
 *    open), 0 to switch it off, at most 1024, default 64. Per graph with
 *    t' = min(far_trim, n / 64) >= 1: each axis is cut into 2048 equal bins
 *    over the bounding box (bin = floor((v - v_min) * 2048 / width) in FP64,
 *    the last bin closed); lo / hi are the bins of the (t'+1)-th smallest /
 *    largest coordinate. When the region of the bins [lo, hi] on both axes
 *    has a larger side of at most half the bounding box's, the grid covers
 *    that region and the points outside it (at most 4 t') are far points:
 *    between a far point and a core point the kernel is interpolated in the
 *    core point's argument only (the far point adds its charges at the nodes
 *    before the gather; its own sums run over the node charges), far points
 *    meet each other exactly. Otherwise the grid covers the bounding box.
 *  min_intervals >= 1, max_intervals a power of two in [min_intervals, 1024]
 *    (default 512). Above 512 every evaluation also launches the transform
 *    kernels of FFT length 6144 (75 KB of LDS per block; TSNET_EINVAL where
 *    the device cannot give that).
 *  Evaluation workspace: a single graph holds grid buffers for a
 *  max_intervals grid (about 2.4 GB at 1024, 600 MB at 512, 9.5 MB at 64).
 *  A batch's grid
 *  buffers are pools with every graph at its own offset, sized by the first
 *  evaluation (which waits once for its grid plan) at four times what its
 *  grids need, at most max_intervals grids in every graph; when a later plan
 *  needs more, the evaluation that finds the pools short halves its largest
 *  grids until they fit (TSNET_STATUS_WORKSPACE and GRID_CAPPED) and the
 *  pools grow before the next evaluation (except under stream capture).
 *  nodes_per_interval: interpolation points per box and axis; must be 3.
 *  attract_layout: TSNET_ATTRACT_*. The tiled layout is a second copy of P
 *    (8 bytes per nonzero) made on the first evaluation that needs it, or in
 *    tsnet_build_P / tsnet_P_from_host when the automatic choice picks it; it
 *    supports up to about 5.8 million vertices (TSNET_EINVAL beyond). Both
 *    layouts compute the same sums in different orders (FP32 results differ
 *    by rounding only).
 *  repulsion, entropy: TSNET_TERMS_*, the method of each sum. Both
 *    interpolated is L-tsNET (Algorithm 3); interpolated repulsion with the
 *    quadtree entropy is FIt-tsNET (Algorithm 2); both by quadtree is
 *    BH-tsNET (Algorithm 1). The quadtree is rebuilt on every evaluation:
 *    per graph, the bounding square split into 2^32 cells per axis (cell of a
 *    coordinate = floor((x - x_min) 2^32 / side) in FP64), points ordered by
 *    the interleaved cell bits (y above x) and then by id, a node per
 *    non-empty 2-bit prefix below a node with two or more points, leaves at
 *    one point or level 32. For point i a node of width w is a summary of
 *    its points (their count at their FP64 centre of mass c) when
 *    w^2 < theta^2 ||X_i - c||^2, tested in FP64; leaves are summed point by
 *    point; the terms are summed in FP32. The tree needs up to 33 n + 1
 *    nodes of 32 bytes, allocated on first use: n at most 65,075,262
 *    (TSNET_EINVAL beyond).
 *  theta: the opening threshold, in (0, 0.7] when a quadtree is used (then a
 *    node holding X_i is never a summary).
 */
typedef struct {
  double  lambda_kl;
  double  lambda_c;
  double  lambda_r;
  double  eps_r;
  double  interval_width;
  int32_t min_intervals;
  int32_t max_intervals;
  int32_t nodes_per_interval;
  int32_t attract_layout;
  int32_t repulsion;
  int32_t entropy;
  double  theta;
  int32_t far_trim;
  int32_t reserved;
} tsnet_params;

/*
 * Vertex move (the last step of the loop of Algorithm 3; the paper names no
 * optimiser): gains <- gains + gain_up where sign(g) != sign(update), else
 * gains * gain_down, floored at min_gain; update <- mu * update - eta * gains * g;
 * X <- X + update. mu = momentum_early for iter < momentum_switch_iter, else
 * momentum_late. eta <= 0 selects max(200, n_g / 12) per graph.
 */
typedef struct {
  double  eta;
  double  momentum_early;
  double  momentum_late;
  double  min_gain;
  double  gain_up;
  double  gain_down;
  int32_t momentum_switch_iter;
  int32_t reserved;
} tsnet_step_params;

/* Defaults: 1, 1.2, 0.01, 0.05, h = 0.25, 50..512 intervals, 3 nodes. */
void tsnet_default_params(tsnet_params* p);
/* Defaults: eta <= 0 (per-graph rule), 0.5 / 0.8 switching at 250, 0.01, 0.2, 0.8. */
void tsnet_default_step_params(tsnet_step_params* p);

/* Create a context on HIP device `device` (made current for the call). */
int tsnet_ctx_create(tsnet_ctx* out, int device);
/* Synchronous; frees everything the context owns. NULL is accepted.
 * TSNET_EINVAL (and nothing freed) while a problem made in it is alive:
 * free every tsnet_P of the context first. */
int tsnet_ctx_destroy(tsnet_ctx ctx);

/*
 * C0 of Algorithm 3: build the symmetric affinities P of a graph batch.
 *  For every vertex, a breadth-first search stops once k other vertices are
 *  visited (Sec. 3.1), ties at equal hop distance broken by a reproducible
 *  key (tie_mode, tie_seed); p_{j|i} follows Eq. (3) with the bandwidth of
 *  each row set by FP64 bisection to perplexity `perplexity`; rows that
 *  cannot reach it take the limiting uniform distribution and set a status
 *  bit; P = (p_{j|i} + p_{i|j}) / (2 n'_g) per Eq. (2), with n'_g the number of
 *  non-empty rows of the graph, over the union of the selected pairs and
 *  their transposes.
 *  indptr [n+1] int64, indices [num_arcs] int32: device CSR of an undirected
 *    simple graph (every edge stored in both rows, rows sorted ascending, no
 *    self loops, no arc between different graphs). Checked on the device;
 *    a violation returns TSNET_EINVAL.
 *  graph_offsets_host: host int32 [num_graphs+1], 0 = first, n = last; NULL
 *    means one graph (num_graphs must then be 1).
 *  k: neighbours per vertex; 0 selects floor(3 * perplexity). 1 <= k <= 1024.
 *  Synchronous (reads back the number of nonzeros). On success *out owns
 *  all device memory of the problem; free it with tsnet_P_free.
 */
int tsnet_build_P(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices,
                  int32_t n, int64_t num_arcs,
                  const int32_t* graph_offsets_host, int32_t num_graphs,
                  double perplexity, int32_t k, uint64_t tie_seed, int32_t tie_mode,
                  tsnet_P* out, void* stream);

/*
 * Pivot MDS settings (tsnet_pmds).
 *  pivots: pivots per graph, 1..128 (a graph with fewer vertices uses all of
 *    them); at least 2 are needed for a non-zero layout.
 *  seed: picks each graph's first pivot.
 *  scale: standard deviation of the first axis of each graph's layout (the
 *    second axis takes the same factor), > 0.
 */
typedef struct {
  int32_t  pivots;
  uint64_t seed;
  double   scale;
} tsnet_pmds_params;

/* Defaults: 50 pivots, seed 0, scale 1e-2 (the spread of the random start). */
void tsnet_default_pmds_params(tsnet_pmds_params* p);

/*
 * Starting layout of Algorithms 1-3 (Sec. 3): Pivot MDS, as tsNET* uses
 * (Sec. 2.1, Sec. 4.1), the eigensolver method of Brandes and Pich. The paper
 * gives no settings; per graph of the batch this computes:
 *  - k_g = min(pivots, n_g) pivots by max-min hop distance, the first at local
 *    index mix64(seed ^ g) mod n_g (SplitMix64 finaliser), ties to the smallest
 *    id, an unreachable vertex counting as infinitely far;
 *  - full BFS hop distances from each pivot, a pair without a path taking 1 +
 *    the graph's largest finite distance;
 *  - C = the double-centred squared distances (n_g x k_g, FP64), the two
 *    leading eigenvectors e1, e2 of C^T C (each signed so that
 *    sum_j (j + 1) e_j > 0 over the pivot order), and X = C [e1 e2] scaled so
 *    that the first axis has standard deviation scale. Fewer than two pivots
 *    give zeros.
 *  indptr, indices, n, num_arcs, graph_offsets_host, num_graphs: the graph
 *    batch as in tsnet_build_P (checked the same way; TSNET_EINVAL if bad).
 *  X: device float [n][2], written. pivots: device int32 [num_graphs][pivots]
 *    (-1 past a graph's k_g) or NULL. eig_host: host double [num_graphs][2]
 *    (lambda1, lambda2 of C^T C) or NULL. levels_host: host, total BFS levels
 *    run, or NULL.
 *  Synchronous: the host reads each BFS level's frontier size and solves the
 *  small eigenproblems (cyclic Jacobi). Device workspace of about
 *  4 n min(pivots, n) bytes is allocated for the call and freed.
 */
int tsnet_pmds(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices, int32_t n,
               int64_t num_arcs, const int32_t* graph_offsets_host, int32_t num_graphs,
               const tsnet_pmds_params* prm, float* X, int32_t* pivots, double* eig_host,
               int32_t* levels_host, void* stream);

/*
 * One stage of a layout run: `iterations` gradient + step iterations with
 * `params` (cost weights, interpolation settings and the L-tsNET / FIt-tsNET
 * / BH-tsNET choice of the sums).
 */
typedef struct {
  int32_t      iterations;
  int32_t      reserved;       /* 0 */
  tsnet_params params;
} tsnet_stage;

/*
 * The gradient-descent loop of Algorithms 1-3 over a table of stages: for
 * each stage and each of its iterations, tsnet_grad with the stage's
 * parameters, then tsnet_step with iteration number first_iter + (iterations
 * run so far). The paper changes the multipliers lambda between stages of
 * the descent (Sec. 2.1) without giving values; a two-stage table expresses
 * such a schedule. X, update, gains: device float [n][2], updated in place;
 * G: device float [n][2] (the last gradient); Z: device double [num_graphs]
 * (the last Z) or NULL. Every stage's parameters are checked before anything
 * is enqueued (TSNET_EINVAL: the message names the stage). Enqueues only, on
 * the stream, the same kernels in the same order as the per-iteration calls
 * (results are bit-identical to them); run one gradient first if the run is
 * to be captured into a graph (the first evaluation sizes the workspace).
 */
int tsnet_run(tsnet_ctx ctx, tsnet_P P, float* X, float* update, float* gains, float* G, double* Z,
              const tsnet_stage* stages, int32_t num_stages, int32_t first_iter,
              const tsnet_step_params* sp, void* stream);

/*
 * Neighbourhood preservation with r = 2 (Sec. 4.3.1), the first quality
 * measure of the experiments. The paper gives the formula; the readings are:
 *  - N_G(v): the vertices 1 or 2 hops from v, v excluded; k_v = |N_G(v)|;
 *  - N_D(v): the k_v vertices of v's own graph nearest to v in the layout, v
 *    excluded, ranked by the FP32 squared distance dx*dx + dy*dy (dx = x_w -
 *    x_v, dy = y_w - y_v, each operation rounded on its own, no fused
 *    multiply-add), equal distances by increasing id;
 *  - hits_v = |N_G(v) & N_D(v)|, so the Jaccard ratio is hits / (2k - hits);
 *  - NP of a graph: the mean of that ratio over its evaluated vertices with
 *    k_v > 0 (NaN if there are none).
 *  indptr, indices, n, num_arcs, graph_offsets_host, num_graphs: the graph
 *    batch as in tsnet_build_P (checked the same way; TSNET_EINVAL if bad).
 *  X: device float [n][2], finite (TSNET_EINVAL otherwise).
 *  vertices: device int32 [num_vertices], strictly increasing vertex ids to
 *    evaluate (TSNET_EINVAL if not), or NULL for every vertex (num_vertices
 *    must then be n).
 *  ball, hits: device int32 [num_vertices], written: k_v and hits_v of each
 *    evaluated vertex, exact integers.
 *  np_host: host double [num_graphs] or NULL.
 *  Synchronous. Device workspace (grid, sorted points, per-worker bitmaps of
 *  the largest graph's vertices, at most about 512 MB of them) is allocated
 *  for the call and freed.
 */
int tsnet_np(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices, int32_t n,
             int64_t num_arcs, const int32_t* graph_offsets_host, int32_t num_graphs,
             const float* X, const int32_t* vertices, int32_t num_vertices, int32_t* ball,
             int32_t* hits, double* np_host, void* stream);

/*
 * Stress (Sec. 4.3.2), the second quality measure, over the ordered pairs
 * (s, j) with s a source, j != s reachable from s, d the hop distance and e
 * the Euclidean layout distance (FP64 from the FP32 coordinates). Per graph
 * g, sums_host[6g + q] holds:
 *  q = 0: the number of pairs; 1: S1 = sum (1 - e/d)^2 (the paper's term
 *  ((d - e)/d)^2); 2: B = sum e/d; 3: C = sum (e/d)^2;
 *  q = 4: the stress S1 / pairs (NaN without pairs);
 *  q = 5: the stress of the layout scaled by alpha = B / C, the factor that
 *  minimises it: (pairs - B^2 / C) / pairs (q = 4's value if C = 0).
 * With every vertex of a connected graph a source the pairs are its n(n-1)
 * ordered pairs and q = 4 is the paper's stress; a sample of sources
 * estimates it. Pairs without a path are left out.
 *  indptr ... num_graphs, X: as in tsnet_np.
 *  sources: device int32 [num_sources] (any order, repeats count again);
 *    an id out of range gives TSNET_EINVAL.
 *  sums_host: host double [num_graphs][6], written. levels_host: host, BFS
 *    levels run in all, or NULL.
 *  Synchronous: the host reads after each BFS level whether it reached a new
 *  vertex. Device workspace of about 48 n bytes is allocated and freed.
 */
int tsnet_stress(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices, int32_t n,
                 int64_t num_arcs, const int32_t* graph_offsets_host, int32_t num_graphs,
                 const float* X, const int32_t* sources, int32_t num_sources, double* sums_host,
                 int32_t* levels_host, void* stream);

/*
 * Make a problem from a host CSR of P (rows sorted, values >= 0, symmetric by
 * contract, not checked). For tests and callers that build P elsewhere.
 * Synchronous. beta/status/conditional rows are absent for such a problem.
 */
int tsnet_P_from_host(tsnet_ctx ctx, int32_t n, const int64_t* rowptr_host,
                      const int32_t* col_host, const float* val_host,
                      const int32_t* graph_offsets_host, int32_t num_graphs, tsnet_P* out);

/* Sizes of a problem (host outputs; any may be NULL). */
int tsnet_P_info(tsnet_P P, int64_t* n, int64_t* nnz, int32_t* num_graphs, int32_t* k);

/*
 * Synchronous copy-out of P and of the conditional rows. Every pointer may be
 * host or device memory, or NULL to skip it. Sizes: rowptr [n+1], col/val
 * [nnz], beta [n] (+inf for rows saturated from above), status [n]
 * (0 ok, 1 low, 2 high, 3 empty), cond_len [n], cond_nbr/cond_dist [n*k]
 * (row i holds cond_len[i] neighbours sorted by (hop distance, tie key, id)).
 * Returns TSNET_EINVAL if conditional data is asked of a problem made by
 * tsnet_P_from_host.
 */
int tsnet_P_export(tsnet_P P, int64_t* rowptr, int32_t* col, float* val, double* beta,
                   int8_t* status, int32_t* cond_len, int32_t* cond_nbr, uint16_t* cond_dist);

/* Synchronous; frees the problem. NULL is accepted. */
int tsnet_P_free(tsnet_P P);

/*
 * One evaluation of dC/dX (Eq. 1 with Eq. 6 and Eq. 8), FP32 interpolation
 * path: G_i = 4 lambda_kl (F_attr,i - F_rep,i / Z) + (lambda_c / n_g) X_i
 *             - (lambda_r / n_g^2) F_ent,i.
 *  X [n][2] float in, G [n][2] float out (may not alias X).
 *  Z_out: device double [num_graphs] or NULL.
 * Non-finite X sets TSNET_STATUS_NONFINITE and yields non-finite G.
 */
int tsnet_grad(tsnet_ctx ctx, tsnet_P P, const float* X, const tsnet_params* prm,
               float* G, double* Z_out, void* stream);

/*
 * Same evaluation, also writing its parts (each output may be NULL):
 *  F_attr, F_rep, F_ent [n][2] float as in the formula above; Z_i [n] float,
 *  the interpolated sum_{j != i} (1 + ||X_i - X_j||^2)^-1.
 */
int tsnet_grad_terms(tsnet_ctx ctx, tsnet_P P, const float* X, const tsnet_params* prm,
                     float* G, double* Z_out, float* F_attr, float* F_rep, float* F_ent,
                     float* Z_i, void* stream);

/*
 * The vertex move, in place on X, update, gains ([n][2] float each) with the
 * gradient G of the current iteration `iter` (0-based).
 */
int tsnet_step(tsnet_ctx ctx, tsnet_P P, float* X, float* update, float* gains,
               const float* G, const tsnet_step_params* sp, int32_t iter, void* stream);

/*
 * The cost of Eq. (1) with the entropy as -lambda_r / (4 n^2) sum ln(eps + r^2)
 * (the form whose gradient is Eq. 8), evaluated with the same interpolation:
 *  cost: device double [num_graphs][4] = {C_KL, C_CMP, C_ENT, total}.
 */
int tsnet_cost(tsnet_ctx ctx, tsnet_P P, const float* X, const tsnet_params* prm,
               double* cost, void* stream);

/*
 * Exact all-pairs FP64 gradient (the O(n^2) tsNET evaluation over the same
 * sparse P), the comparison baseline: Eq. (6) for the KL part with the
 * normaliser Z of Sec. 2.1 summed over every pair, the entropy part of
 * Eq. (8) pair by pair and the compression derivative, assembled as in
 * tsnet_grad. X, G [n][2] double.
 *  rows: NULL for every vertex, else device int32 [nrows] vertex ids; G is
 *    then [nrows][2] and only those rows are evaluated (Z is still summed over
 *    all pairs of each graph).
 *  terms: NULL or device double [nrows or n][7] = {F_attr x,y, F_rep x,y,
 *    F_ent x,y, Z_i}.
 *  Z_out: NULL or device double [num_graphs].
 */
int tsnet_grad_direct_f64(tsnet_ctx ctx, tsnet_P P, const double* X, const tsnet_params* prm,
                          double* G, double* Z_out, const int32_t* rows, int32_t nrows,
                          double* terms, void* stream);

/*
 * tsnet_grad_direct_f64 for callers that cannot allocate device memory: code
 * being captured into a HIP graph, tight serving loops, harnesses that forbid
 * allocation. Same arguments, results and kernels (bit-identical output);
 * the per-row pair sums go to a file-scope device array of 2^21 doubles
 * (16 MiB) that every GPU the library runs on holds until the process ends,
 * instead of a buffer the problem allocates on first use. It calls no
 * allocating routine and records no stage timing.
 *  Limit: 5 * (n + nrows) <= 2^21 with rows, 5 * n <= 2^21 without (n at
 *    most 419,430 for every row); larger calls fail with TSNET_EINVAL before
 *    anything is enqueued.
 *  All calls on one GPU share that GPU's array, which keeps the last call's
 *  contents: calls that overlap on one GPU (other streams, other threads,
 *  other contexts) race and must be ordered by the caller. Nothing in the
 *  array needs to start at zero (every value is written before it is read
 *  within a call).
 */
int tsnet_grad_direct_f64_static(tsnet_ctx ctx, tsnet_P P, const double* X,
                                 const tsnet_params* prm, double* G, double* Z_out,
                                 const int32_t* rows, int32_t nrows, double* terms, void* stream);

/*
 * Grid of the most recent tsnet_grad / tsnet_cost on P, per graph (host
 * arrays [num_graphs], any may be NULL): intervals per axis, box side,
 * lower-left corner, number of far points set apart (far_trim). Synchronous.
 */
int tsnet_grid_info(tsnet_P P, int32_t* n_intervals, float* box_side, float* x0, float* y0,
                    int32_t* far_points);

/*
 * Device bytes of P's grid workspace (host-side bookkeeping, no GPU call):
 * the grid buffers (charges, spectra, products, potentials), the box offsets
 * and the far-point bin counts. A single graph holds grid buffers for a
 * max_intervals grid; a batch holds pools sized from its plans (four times
 * the first evaluation's needs, at most max_intervals grids in every graph).
 */
int tsnet_workspace_bytes(tsnet_P P, size_t* bytes_host);

/* Synchronous: OR of the TSNET_STATUS_* bits raised since the last call; clears them. */
int tsnet_status(tsnet_ctx ctx, uint32_t* flags_host);

/*
 * Per-stage GPU timing for profiling. stage_mask has bit s set for every
 * stage s (0 <= s < tsnet_stage_count()) to be bracketed by HIP events on the
 * call's stream; 0 turns timing off. tsnet_stage_times (synchronous) returns
 * accumulated milliseconds and call counts per stage ([tsnet_stage_count()]
 * host arrays, either may be NULL) and resets them; names via
 * tsnet_stage_name. The Z reduction runs inside the gather kernel, so the
 * "z_reduce" stage (kept so stage ids stay stable) records no calls.
 */
int tsnet_set_timing(tsnet_ctx ctx, uint32_t stage_mask);
int tsnet_stage_count(void);
const char* tsnet_stage_name(int stage);
int tsnet_stage_times(tsnet_ctx ctx, double* ms_host, int64_t* calls_host);

/* Message of the calling thread's most recent failure ("" if none). */
const char* tsnet_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TSNET_H */
