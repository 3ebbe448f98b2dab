/*
 * tsgne.h -- C-ABI of the MI355X (gfx950) t-SGNE optimisation loop.
 *
 * The library turns a graph G = (V, E) (undirected, unweighted, |V| = n) and a
 * node embedding X = {x_i in R^d} into a 2-D layout Y = {y_i in R^2}, the
 * dimension-reduction half of GD = DR o GE (Li, Xiao, Zhou, "Efficiently
 * Visualizing Large Graphs", arXiv 2310.11186, section 2, eq. (1)).  The
 * affinities P follow section 2.1, eqs. (2)-(3), restricted to each node's
 * graph neighbours as t-SGNE prescribes (section 2.2, eq. (7)); the layout
 * minimises KL(P || Q) of eq. (5) with the Student-t Q of eq. (4).
 *
 * Conventions for every call:
 *  - Pointers ending in _d are device pointers (HBM of the current HIP
 *    device); pointers ending in _h are host pointers.  The caller owns every
 *    pointer it passes; the library only reads or writes it during the call
 *    (device writes complete in stream order).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it.  Calls marked "synchronising" block until
 *    their work on `stream` has finished.
 *  - Layouts: X is float32 [n][d] row-major; Y, upd, gains and grad are float32
 *    [n][2] (x, y interleaved); the CSR is int32 row_ptr[n+1], col[nnz].
 *  - Every call returns a tsgne_status; on failure tsgne_last_error() gives a
 *    message (thread-local, valid until the next call on that thread).  No C++
 *    exception crosses this boundary.  Errors raised by the device inside an
 *    asynchronous call surface at the next synchronising call.
 *  - A tsgne_graph* is owned by the library; release it with tsgne_graph_free.
 *    Calls on one graph must not overlap (they share its workspace); different
 *    graphs may be used concurrently from different threads.
 *  - Device memory of the step workspace (allocated on the first step,
 *    gradient or run): the repulsion partials take 8 * n * nb bytes, nb =
 *    ceil(n / (64 * tile_rows)) (about 0.8 GB at 300K nodes, 31 GB at 2M with
 *    16 rows per lane), plus about 40 bytes per node and 8 per tile; a graph
 *    whose workspace does not fit fails with E_NOMEM.
 */
#ifndef TSGNE_H
#define TSGNE_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define TSGNE_API __attribute__((visibility("default")))
#else
#define TSGNE_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tsgne_status;
#define TSGNE_OK 0
#define TSGNE_E_INVAL (-1)     /* bad argument: null pointer, size, parameter */
#define TSGNE_E_GRAPH (-2)     /* CSR not canonical (sorted, no self-loops) or not symmetric */
#define TSGNE_E_NOMEM (-3)     /* device or host allocation failed */
#define TSGNE_E_DEVICE (-4)    /* a HIP runtime call failed */
#define TSGNE_E_NONFINITE (-5) /* a non-finite value appeared in the layout */
#define TSGNE_E_BUSY (-6)      /* resource busy (queue full, request still running) */
#define TSGNE_E_CANCELLED (-7) /* the request was cancelled */

/* Precision modes of the per-step arithmetic. */
#define TSGNE_PREC_SPLIT 0 /* FP32 pair arithmetic; FP64 for Z, cross-tile force sums, KL */
#define TSGNE_PREC_FP32 1  /* everything FP32 (reported for comparison) */

/* Repulsion kernel choice. */
#define TSGNE_REPULSION_AUTO 0
#define TSGNE_REPULSION_DIRECT 1    /* every ordered pair computed by its row's lane */
#define TSGNE_REPULSION_SYMMETRIC 2 /* each unordered pair once, w_ij = w_ji shared */

/*
 * Optimiser parameters.  The paper names the objective (eq. (5)) but no
 * optimiser; these are the usual t-SNE gradient-descent settings: early
 * exaggeration of P, momentum, per-coordinate gains.
 */
typedef struct tsgne_params {
  float early_exaggeration;   /* alpha applied to P while t < exaggeration_iters (default 12) */
  int32_t exaggeration_iters; /* default 250; set n_iter/4 for other lengths */
  float learning_rate;        /* eta; <= 0 selects max(n / (4 * early_exaggeration), 50) */
  float momentum_early;       /* momentum while t < exaggeration_iters (default 0.5) */
  float momentum_late;        /* momentum afterwards (default 0.8) */
  float min_gain;             /* lower clamp of the gains (default 0.01) */
  int32_t precision;          /* TSGNE_PREC_SPLIT (default) or TSGNE_PREC_FP32 */
  int32_t kl_every;           /* tsgne_run: record KL after every kl_every-th step; 0 = off */
  int32_t repulsion;          /* TSGNE_REPULSION_* (default AUTO = SYMMETRIC) */
  int32_t tile_rows;          /* rows per lane of the repulsion tile: 1, 2, 4, 8, 12, 14, 15, 16 or 0 = auto */
} tsgne_params;

typedef struct tsgne_graph tsgne_graph;

/* Fills *p with the defaults listed above. */
TSGNE_API void tsgne_params_default(tsgne_params* p);

/*
 * The repulsion plan a graph of n nodes gets for tile_rows (0 = automatic)
 * and repulsion (TSGNE_REPULSION_*), without a device: *tile_rows_out the
 * rows per lane, *tiles_out the tiles per step (the tile triangle for the
 * symmetric kernel, the whole square for the direct one), *partial_bytes_out
 * the device bytes of the step's repulsion partials (8 * n * nb).  Any output
 * may be NULL.  Host only.  Errors: E_INVAL (n < 1, unsupported tile_rows).
 */
TSGNE_API tsgne_status tsgne_repulsion_plan(int32_t n, int32_t tile_rows, int32_t repulsion, int32_t* tile_rows_out,
                                            int64_t* tiles_out, int64_t* partial_bytes_out);

/* Message of the last failure on this thread ("" if none). */
TSGNE_API const char* tsgne_last_error(void);

/* Static name of a status code. */
TSGNE_API const char* tsgne_status_string(tsgne_status s);

/*
 * Host helper: canonical symmetric CSR of an undirected edge list (section 2:
 * G is undirected and unweighted).  uv_h holds m pairs (u, v) as int32[m][2];
 * self-loops are dropped, each edge is stored both ways, columns are sorted
 * ascending and repeats removed.  row_ptr_h must hold n+1 entries and col_h
 * 2*m.  *nnz_out receives the number of stored entries.
 * Errors: E_INVAL for null pointers, n < 0, m < 0, an endpoint outside [0, n)
 * or a result with 2^31 or more entries.
 */
TSGNE_API tsgne_status tsgne_csr_from_edges(int32_t n, int64_t m, const int32_t* uv_h, int32_t* row_ptr_h, int32_t* col_h,
                                  int64_t* nnz_out);

/*
 * The t-SGNE neighbourhood graph G_knn,G of section 2.2, eq. (7): nodes i and
 * j are joined when one is among the first k nearest neighbours of the other
 * on G, nearest by breadth-first search.  Reading: the first k neighbours of i
 * are the k smallest nodes j != i under (hop distance from i, node id), fewer
 * when i's component is smaller.  The result can be passed to tsgne_build_P in
 * place of G's own CSR.
 *   n, nnz, row_ptr_d, col_d -- G as a canonical symmetric CSR (device), as
 *                               for tsgne_build_P
 *   k                        -- 1 .. 256
 *   knn_row_ptr_d            -- int32[n+1] (device, written)
 *   knn_col_d                -- int32[knn_capacity] (device, written); 2*n*k
 *                               always suffices
 *   *knn_nnz                 -- number of stored entries of the result (also
 *                               set when the capacity is too small)
 * Synchronising.  Errors: E_INVAL (bad sizes, k, capacity too small),
 * E_GRAPH (input CSR not canonical/symmetric), E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_knn_graph(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d,
                                       int32_t k, int32_t* knn_row_ptr_d, int32_t* knn_col_d, int64_t knn_capacity,
                                       int64_t* knn_nnz, void* stream);

/*
 * The ShortestPath graph embedding of section 2.3, eq. (8): X[i][j] is the
 * hop distance between node i and target t_j when it is at most l0, and
 * l0 + 1 when it is larger or t_j cannot be reached from i.  Readings: the
 * condition of eq. (8) is on d_ij, and the equation (at most l0) is
 * followed.  The paper picks the d targets at random; the caller passes them.
 * X can be passed to tsgne_build_P as the node embedding.
 *   n, nnz, row_ptr_d, col_d -- G as a canonical symmetric CSR (device), as
 *                               for tsgne_build_P
 *   d                        -- number of targets, 1 .. 256
 *   targets_d                -- int32[d] (device) node ids in [0, n);
 *                               repeats allowed
 *   l0                       -- threshold; a negative value selects the
 *                               paper's default sqrt(|E|), |E| = nnz / 2
 *   X_d                      -- float32[n][d] row-major (device, written)
 *   levels_out               -- nullable; receives the number of search
 *                               levels launched (at most floor(l0))
 * Synchronising.  Errors: E_INVAL (bad sizes, NaN l0, a target outside
 * [0, n)), E_GRAPH (CSR not canonical/symmetric), E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_shortest_path_embedding(int32_t n, int64_t nnz, const int32_t* row_ptr_d,
                                                     const int32_t* col_d, int32_t d, const int32_t* targets_d,
                                                     double l0, float* X_d, int32_t* levels_out, void* stream);

/*
 * Layout quality (sections 2.5-2.6).  The three calls below are
 * synchronising and leave every input unchanged.
 *
 * tsgne_kmeans: the clustering of the layout used for the NMI of section
 * 2.5, which the paper calls kNN clustering with k set to the number of graph
 * clusters; read as Lloyd's k-means.  The layout is mapped onto a 2^24 x 2^24
 * grid over its bounding box (q = min(floor((y - lo) / (hi - lo) * 2^24),
 * 2^24 - 1), 0 on a flat axis) so that every decision is reproducible: each
 * pass assigns every point to the nearest centre (squared distance in FP64,
 * ties to the lower index) and, unless no label changed, moves each
 * non-empty cluster's centre to the exact mean of its points; an empty
 * cluster keeps its centre.
 *   n, Y_d      -- float32[n][2] layout (device), n >= 1
 *   k           -- 1 .. 1024 clusters
 *   seeds_d     -- int32[k] (device): the initial centres are the points at
 *                  these node indices (the caller draws them)
 *   max_iter    -- at most this many passes (>= 1)
 *   labels_d    -- int32[n] (device, written): cluster of each node
 *   iters_out   -- nullable: passes made (the last one changed nothing,
 *                  unless max_iter was reached)
 * Errors: E_INVAL (sizes, a seed outside [0, n)), E_NONFINITE (a
 * non-finite coordinate), E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_kmeans(int32_t n, const float* Y_d, int32_t k, const int32_t* seeds_d, int32_t max_iter,
                                    int32_t* labels_d, int32_t* iters_out, void* stream);

/*
 * tsgne_nmi: normalised mutual information of two labelings of n nodes
 * (section 2.5, eq. (11)): 2 I(A;B) / (H(A) + H(B)), natural logarithms;
 * identical partitions give 1, and two single-cluster labelings give 1.
 *   a_d, b_d -- int32[n] (device), labels in [0, ka) and [0, kb)
 *   ka, kb   -- label counts, ka * kb <= 2^26
 *   nmi_out  -- host double (written)
 * Errors: E_INVAL (sizes, a label out of range), E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_nmi(int32_t n, const int32_t* a_d, int32_t ka, const int32_t* b_d, int32_t kb,
                                 double* nmi_out, void* stream);

/*
 * tsgne_aq: aesthetic quality of a layout (section 2.6, eqs. (12)-(14)): the
 * bounding box is cut into grid x grid cells of width (Xmax - Xmin) / grid
 * and height (Ymax - Ymin) / grid; a cell is good when the largest fraction
 * of its points sharing one label exceeds p; AQ = good cells / grid^2.
 * Readings: points on the upper edge belong to the last cell, an empty cell
 * is not good, a flat axis puts every point in its first cell.
 *   Y_d      -- float32[n][2] layout (device)
 *   labels_d -- int32[n] (device) in [0, n_labels) (e.g. graph communities)
 *   grid     -- 1 .. 4096, grid^2 * n_labels <= 2^28
 *   p        -- threshold
 *   aq_out   -- host double (written)
 * Errors: E_INVAL, E_NONFINITE, E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_aq(int32_t n, const float* Y_d, const int32_t* labels_d, int32_t n_labels, int32_t grid,
                                double p, double* aq_out, void* stream);

/*
 * Node renumbering for memory locality.  By the premise of t-SGNE (section
 * 2.2) nodes close in the graph are close in R^d, so numbering the nodes
 * along a space-filling curve of the embedding puts most graph neighbours at
 * nearby ids, and the position gathers of the attraction stay within a small
 * window of Y.  Optional: results in the new numbering map back to the
 * caller's with tsgne_permute_rows(..., inverse = 1, ...).
 *
 * tsgne_locality_order: perm_d[r] = the node of rank r in the Morton
 * (Z-order) of the leading m = min(d, 8) coordinates of X, each quantised to
 * b = 64 / m bits over its own range (q = min(floor((x - lo) / (hi - lo) *
 * 2^b), 2^b - 1), 0 on a flat axis) and interleaved from the top bit down,
 * coordinate 0 first; ties in node id order.
 *   X_d    -- float32[n][d] (device);  perm_d -- int32[n] (device, written)
 * Synchronising.  Errors: E_INVAL, E_NONFINITE, E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_locality_order(int32_t n, const float* X_d, int32_t d, int32_t* perm_d, void* stream);

/*
 * tsgne_permute_graph: the graph renumbered by perm (new node r = old node
 * perm[r]): (r, s) is an edge iff (perm[r], perm[s]) is one.  The input is a
 * canonical symmetric CSR (as for tsgne_build_P); the output is one too.
 *   perm_d        -- int32[n] (device), a permutation of [0, n)
 *   out_row_ptr_d -- int32[n+1] (device, written); out_col_d -- int32[nnz]
 * Synchronising.  Errors: E_INVAL (sizes, perm not a permutation), E_GRAPH,
 * E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_permute_graph(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d,
                                           const int32_t* perm_d, int32_t* out_row_ptr_d, int32_t* out_col_d,
                                           void* stream);

/*
 * tsgne_permute_rows: rows of row_bytes bytes (a multiple of 4) of a
 * row-major device array: dst row r = src row perm[r] (inverse = 0, e.g. X
 * or Y0 into the new numbering), or dst row perm[r] = src row r (inverse =
 * 1, e.g. a layout back into the old numbering).  src and dst must not
 * overlap.  Asynchronous on the stream.  Errors: E_INVAL, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_permute_rows(int32_t n, int32_t row_bytes, const void* src_d, const int32_t* perm_d,
                                          int32_t inverse, void* dst_d, void* stream);

/*
 * Builds the joint affinities P of eq. (3) from the conditional affinities of
 * eq. (2) over each node's graph neighbours (section 2.2), with the bandwidth
 * of each row set by bisection so that its perplexity equals `perplexity`
 * (section 2.1, entropy in nats against log(perplexity)).
 *   n, nnz       -- number of nodes and of CSR entries (nnz < 2^31)
 *   row_ptr_d    -- int32[n+1], col_d int32[nnz]: canonical symmetric CSR
 *                   (row_ptr[0] = 0, row_ptr[n] = nnz, nondecreasing; columns
 *                   in [0, n), strictly ascending per row, no self-loops,
 *                   (i,j) stored iff (j,i) is)
 *   X_d          -- float32[n][d], d >= 1
 *   perplexity   -- > 1 (the paper's usual range is 5-50, 30 by default)
 * Rows with deg <= perplexity are uniform (the target entropy is out of reach);
 * isolated nodes get empty rows and P is normalised by 2 * (non-isolated
 * nodes) so that it sums to one (eq. (3) writes 2n, which assumes no isolated
 * node).  P is stored as float32 aligned with col, computed in FP64.
 * The inputs are read during the call only: the graph keeps its own copies.
 * Synchronising (the CSR check is read back).  *out receives a new graph.
 * Errors: E_INVAL (null pointer, n < 1, nnz < 0, d < 1, perplexity <= 1 or
 * not finite), E_GRAPH (CSR not canonical or not symmetric), E_NOMEM,
 * E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_build_P(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d, const float* X_d,
                           int32_t d, float perplexity, void* stream, tsgne_graph** out);

/*
 * The approximation of P by random walks of section 2.1, as an alternative to
 * tsgne_build_P: each node starts `walks` walks of `length` steps on G; a step
 * from u goes to the neighbour v with probability proportional to
 * exp(-||x_u - x_v||^2) (read with the minus sign the printed formula lacks;
 * evaluated as exp(-(D_uv - D_min,u)) with D in FP64); p_{j|i} = (walks from
 * i ending at j != i) / walks, and symmetrising as in eq. (3) with the total
 * mass gives P_ij = (c_ij + c_ji) / (2 M), M = walks that do not end at their
 * start.  The returned graph's CSR is the support of the walks (pairs with
 * c_ij + c_ji > 0, canonical and symmetric; at most `length` hops apart) and
 * can be used with every call that takes a tsgne_graph; beta is zero.
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011) with counter
 * (node, walk, step, 0) and key (seed low 32 bits, seed high 32 bits); the
 * uniform is (x0 * 2^21 + (x1 >> 11)) * 2^-53, and the step takes the first
 * CSR entry whose running weight exceeds uniform * row total (the last entry
 * if none does).  A walk from an isolated node stays put.
 *   n, nnz, row_ptr_d, col_d, X_d, d -- as for tsgne_build_P
 *   walks  -- walks per node, >= 1, with 2 * n * walks < 2^31
 *   length -- steps per walk, 1 .. 4096
 *   seed   -- Philox key
 * Synchronising.  Errors: E_INVAL, E_GRAPH (input CSR), E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_build_P_walks(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d,
                                           const float* X_d, int32_t d, int32_t walks, int32_t length, uint64_t seed,
                                           void* stream, tsgne_graph** out);

/*
 * A graph whose joint affinities P are given instead of built: the CSR
 * (row_ptr_h int32[n+1], col_h int32[nnz], host, canonical and symmetric as
 * for tsgne_build_P) and P_h float32[nnz] (host, aligned with col_h) are
 * copied in.  P plays the role of eq. (3)'s joint affinities: it must be
 * finite, non-negative and symmetric entry by entry (p_ij == p_ji bitwise);
 * it should sum to one (not checked).  Meant for checking the optimisation
 * loop on affinities computed elsewhere (e.g. a reference implementation's
 * P rounded to FP32).  The graph's beta (tsgne_graph_export) reads 0.
 * Synchronising.  *out is library-owned; release it with tsgne_graph_free.
 * Errors: E_INVAL (sizes, null pointers, P not finite, negative or not
 * symmetric), E_GRAPH (CSR not canonical or not symmetric), E_NOMEM,
 * E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_graph_from_host_P(int32_t n, int64_t nnz, const int32_t* row_ptr_h, const int32_t* col_h,
                                               const float* P_h, void* stream, tsgne_graph** out);

/* Releases a graph and all device memory it holds.  NULL is accepted. */
TSGNE_API tsgne_status tsgne_graph_free(tsgne_graph* g);

/* Size of a graph: *n nodes, *nnz stored CSR entries (either may be NULL). */
TSGNE_API tsgne_status tsgne_graph_info(const tsgne_graph* g, int32_t* n, int64_t* nnz);

/*
 * Copies the graph's device state to host buffers (any may be NULL):
 * row_ptr_h int32[n+1], col_h int32[nnz], mirror_h int32[nnz] (position of
 * entry (j,i) for entry (i,j)), P_h float32[nnz], beta_h float64[n] (the
 * calibrated 1/(2 sigma_i^2); 0 for uniform rows, +inf for rows uniform over
 * tied nearest neighbours).  Synchronising (on the null stream).
 */
TSGNE_API tsgne_status tsgne_graph_export(const tsgne_graph* g, int32_t* row_ptr_h, int32_t* col_h, int32_t* mirror_h,
                                float* P_h, double* beta_h);

/*
 * Gradient of eq. (5) at Y with P scaled by alpha (early exaggeration):
 *   g_i = 4 * sum_{j != i} (alpha * p_ij - q_ij) * w_ij * (y_i - y_j),
 *   w_ij = (1 + ||y_i - y_j||^2)^-1,  q_ij = w_ij / Z,  Z = sum_{k != l} w_kl
 * (eq. (4)).  Y_d float32[n][2] (read), grad_d float32[n][2] (written),
 * Z_d float64[1] (written; may be NULL).  precision / repulsion / tile_rows are
 * taken from p (NULL = defaults).  Asynchronous.
 * Errors: E_INVAL, E_NOMEM (first use allocates the step workspace), E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_gradient(tsgne_graph* g, const float* Y_d, float alpha, const tsgne_params* p, float* grad_d,
                            double* Z_d, void* stream);

/*
 * The attractive half of the gradient of eq. (5), per row i:
 *   A_i = sum over stored entries j of p_ij * w_ij * (y_i - y_j)
 * (unscaled: the gradient is 4 (alpha A_i - R_i / Z)).  Y_d float32[n][2]
 * (read), A_d float64[n][2] (written; FP32 arithmetic per entry, accumulated
 * in FP64 for TSGNE_PREC_SPLIT, all FP32 for TSGNE_PREC_FP32, stored as
 * float64 either way).  Needs no repulsion workspace.  Asynchronous.
 * Errors: E_INVAL, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_attraction(tsgne_graph* g, const float* Y_d, int32_t precision, double* A_d,
                                        void* stream);

/*
 * One optimisation step at index t: the gradient above with alpha =
 * early_exaggeration if t < exaggeration_iters else 1, then per coordinate
 *   gain <- (g * u < 0) ? gain + 0.2 : 0.8 * gain;  gain <- max(gain, min_gain);
 *   u <- m_t * u - eta * gain * g;  y <- y + u
 * with m_t = momentum_early if t < exaggeration_iters else momentum_late.
 * Y_d, upd_d, gains_d: float32[n][2], updated in place (start with upd = 0,
 * gains = 1).  grad_out_d (nullable) receives g at the input Y; Z_out_d
 * (nullable, float64[1]) receives Z at the input Y.  Asynchronous.
 * Errors: E_INVAL, E_NOMEM (first use allocates the step workspace), E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_step(tsgne_graph* g, float* Y_d, float* upd_d, float* gains_d, int32_t t, const tsgne_params* p,
                        float* grad_out_d, double* Z_out_d, void* stream);

/*
 * n_iter steps t = 0 .. n_iter-1 from the layout in Y_d (float32[n][2], in:
 * Y0, out: final layout), with internal upd (0) and gains (1): the loop that
 * minimises eq. (5).  Equals n_iter calls of tsgne_step bit for bit.  The
 * steps are captured once as a HIP graph of up to 32 steps (the step index
 * lives on the device, which switches exaggeration and momentum at
 * exaggeration_iters) and replayed on `stream`; the host does not touch the
 * layout between steps.  If p->kl_every > 0 and kl_trace_h is not NULL,
 * kl_trace_h[k] receives the KL (eq. (5), unexaggerated P) after step
 * (k+1)*kl_every - 1, for k < n_iter / kl_every: computed inside the next
 * step with the Z that step sums at that layout (FP32-summed Z when
 * p->precision is TSGNE_PREC_FP32), and for the last layout as tsgne_kl does.
 * With phase timing on (tsgne_graph_set_timing) the steps are launched one by
 * one instead, each launch between its own pair of events; the arithmetic is
 * the same.  Synchronising.
 * Errors: E_INVAL, E_NOMEM, E_DEVICE, E_NONFINITE (the final layout holds a
 * NaN or infinity).
 */
TSGNE_API tsgne_status tsgne_run(tsgne_graph* g, float* Y_d, int32_t n_iter, const tsgne_params* p, double* kl_trace_h,
                       void* stream);

/*
 * KL(P || Q) of eq. (5) at layout Y_d (float32[n][2]) with the unexaggerated
 * P, accumulated in FP64.  Q's normaliser Z is recomputed at Y_d by a pass
 * over the repulsion's tiles that forms only the pair weights (FP32 weights,
 * FP64 sums; bitwise the Z a split-precision step sums at Y_d), about half
 * the cost of a force pass.
 * *kl_h receives the value.  Synchronising.
 * Errors: E_INVAL, E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_kl(tsgne_graph* g, const float* Y_d, double* kl_h, void* stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): tsgne_kl without any allocation
 * and without synchronising.  The KL of the layout Y_d (float32[n][2],
 * device) lands in *kl_d (float64, device, caller-owned) in stream order.
 * It runs the kernels of tsgne_kl with the same repulsion plan (the graph's
 * workspace plan, or the automatic one before the graph's first step), so
 * the value is bitwise tsgne_kl's.  Their scratch (tile list, Z partials, KL
 * partials: 16 bytes per repulsion tile plus 8 KiB) lives in a 32 MiB device
 * array that each GPU holds until the process ends (up to about 2 million
 * nodes); a larger graph is refused with E_INVAL and a message giving the
 * size.  Every call on one GPU uses that GPU's one array: calls that overlap
 * on a GPU (different streams, threads or graphs) race and must be ordered
 * by the caller.  Errors: E_INVAL, E_DEVICE (a launch failed).
 */
TSGNE_API tsgne_status tsgne_kl_noalloc(tsgne_graph* g, const float* Y_d, double* kl_d, void* stream);

/*
 * Advances many independent graphs together (the same optimiser as
 * tsgne_run, eqs. (4)-(5) per graph).  graphs[k] / Y_d[k] (float32[n_k][2], in:
 * Y0, out: final layout) for k < count; graph k takes n_iter[k] steps
 * t = 0 .. n_iter[k]-1 with the schedule of p (early exaggeration and
 * momentum switch at p->exaggeration_iters).  Each step is one set of fused
 * launches for the whole batch (repulsion tiles of every graph, per-graph Z,
 * attraction, update), captured once as a HIP graph and replayed.  All graphs
 * use the repulsion tile p->tile_rows (1, 2, 4, 8, 12, 14, 15, 16; 0 = chosen from the batch's
 * total tile count) with symmetric tiles; each graph's arithmetic and
 * reduction order are its own, so its result equals tsgne_run of that graph
 * alone with the same tile_rows and the symmetric repulsion, bit for bit.
 * Graphs must be distinct and on one device; layouts must not alias.  The
 * graphs' step workspaces are re-planned for the batch tile.  stream may be
 * NULL (a private stream is used).  Synchronising.
 * Errors: E_INVAL, E_NOMEM, E_DEVICE, E_NONFINITE (a final layout holds a NaN
 * or infinity).
 */
TSGNE_API tsgne_status tsgne_batch_run(tsgne_graph* const* graphs, float* const* Y_d, const int32_t* n_iter,
                                       int32_t count, const tsgne_params* p, void* stream);

/*
 * Autotuner: times `steps` batched steps (after one warm-up step) of the given
 * graphs for each repulsion tile R in {4, 8, 12, 16} (TSGNE_AUTOTUNE_TILES
 * values), on scratch copies of Y_d (the caller's layouts are only read), and
 * returns the fastest R in *best_tile_rows and, if ms_per_step is not NULL,
 * the average step times (ms) in that order: ms_per_step must hold
 * TSGNE_AUTOTUNE_TILES doubles.  Leaves the graphs' workspaces planned for
 * R = 16.  Synchronising.  Errors: E_INVAL, E_NOMEM, E_DEVICE.
 */
#define TSGNE_AUTOTUNE_TILES 4
TSGNE_API tsgne_status tsgne_autotune(tsgne_graph* const* graphs, const float* const* Y_d, int32_t count,
                                      const tsgne_params* p, int32_t steps, int32_t* best_tile_rows,
                                      double* ms_per_step, void* stream);

/*
 * tsgne_batch_run with a repulsion tile per graph: tile_rows[k] (1, 2, 4, 8,
 * 12, 14, 15, 16; 0 = the single-graph plan's choice for graph k's size).
 * The graphs of each tile size form one batched plan; the plans run side by
 * side (one branch stream each, forked and joined inside each captured chunk
 * of steps).  Graph k's layout equals tsgne_run of it alone with tile_rows[k]
 * and the symmetric repulsion, bit for bit.  Arguments, errors and
 * synchronisation as tsgne_batch_run.
 */
TSGNE_API tsgne_status tsgne_batch_run_tiles(tsgne_graph* const* graphs, float* const* Y_d, const int32_t* n_iter,
                                             const int32_t* tile_rows, int32_t count, const tsgne_params* p,
                                             void* stream);

/*
 * Autotuner of per-graph tiles for tsgne_batch_run_tiles.  Graphs are grouped
 * by size bucket b = floor(log2 n) (b < TSGNE_TILE_BUCKETS); every graph of a
 * bucket takes the bucket's tile.  Buckets the cache fixes keep their tile;
 * for the others it times `steps` batched steps of the whole batch (on scratch
 * copies of Y_d, after a warm-up step) with one tile R in {2, 4, 8, 12, 16} for
 * all of them, keeps the fastest, then, bucket by bucket (heaviest sum of n^2
 * first), tries the other R for that bucket alone and keeps one that makes the
 * batch at least 0.5 % faster.  tile_rows_out[count] receives each graph's
 * tile; *ms_uniform and *ms_tuned (nullable) the ms per step with the best
 * single tile and with the tuned tiles.  cache_path (nullable): a JSON file of
 * {architecture: {bucket: tile rows}} (architecture as the device reports it,
 * e.g. "gfx950"), read first and rewritten with the buckets tuned here.
 * Leaves the graphs' workspaces planned for the last tile tried.
 * Synchronising.  Errors: E_INVAL (also: the cache file cannot be written),
 * E_NOMEM, E_DEVICE.
 */
#define TSGNE_TILE_BUCKETS 32
TSGNE_API tsgne_status tsgne_autotune_tiles(tsgne_graph* const* graphs, const float* const* Y_d, int32_t count,
                                            const tsgne_params* p, int32_t steps, const char* cache_path,
                                            int32_t* tile_rows_out, double* ms_uniform, double* ms_tuned,
                                            void* stream);

/* ------------------------------------------------------------------------
 * Layout server: continuous batching of independent layout requests on the
 * current device.  Requests are copied in at submission and queued; a worker
 * thread admits them while their estimated device footprint fits the budget
 * (building P on admission), advances the active requests in rounds of one
 * batched, graph-captured launch sequence (each request at its own step
 * index), and completes requests that reach n_iter (layout copied out, device
 * memory released).  With round_ms > 0 each round aims at that much GPU time
 * and shares it out as steps (at least 1, at most steps_per_round) by
 * rest_policy: by default requests with little work left go first and long
 * ones run one at a time in submission order, so small requests are not held
 * back by large ones and no large one finishes much later than it would alone
 * in submission order.  With round_ms <= 0 every active request takes
 * steps_per_round steps per round.  Requests of
 * different tile sizes form separate batched plans that run on parallel
 * branches of the round.  Each request's arithmetic depends only on itself
 * and its tile rows: its layout equals tsgne_run of the same graph alone with
 * the symmetric repulsion and tile_rows = the server's tile_rows, or, when
 * that is 0, 8 below 131072 nodes and 0 (the plan's own choice) above (0 for
 * every request when max_active is 1), bit for bit.
 * ------------------------------------------------------------------------ */
typedef struct tsgne_server tsgne_server;

typedef struct tsgne_server_config {
  int64_t hbm_budget;      /* device bytes the server may hold; 0 = 80 % of the free memory */
  int32_t max_active;      /* requests advanced together (default 64) */
  int32_t max_queue;       /* waiting requests before submit returns E_BUSY */
  int32_t steps_per_round; /* most steps a request takes per round (default 512) */
  int32_t tile_rows;       /* repulsion tile rows: 0 (default) = per request, the single-graph plan's choice
                              (its layout equals its own tsgne_run); 1, 2, 4, 8, 12, 14, 15 or 16 = for every
                              request */
  tsgne_params params;     /* optimiser; its exaggeration/momentum schedule applies to every request */
  float round_ms;          /* target GPU time per round (default 25); <= 0: lockstep */
  float oldest_share;      /* TSGNE_SHARE_EQUAL and TSGNE_SHARE_SMALLEST_FIRST: fraction of each round's time
                              given to the oldest active request, the rest shared by rest_policy (default 0.5;
                              0 = the whole round by rest_policy); bounds how far small arrivals can slow the
                              request that has waited longest */
  int32_t rest_policy;     /* how a round is shared: TSGNE_SHARE_SHORT_FIRST (default): requests with at most
                              long_ms of GPU time left take what they need first (least remaining first), and
                              long requests run one at a time in submission order with the rest (the others
                              paused); while a long request runs, the short ones take at most short_share of
                              a round and only as much as the long one is ahead of its estimated finish in
                              the one-at-a-time schedule; with oldest_share: TSGNE_SHARE_EQUAL shares the rest in
                              equal parts, TSGNE_SHARE_SMALLEST_FIRST to the requests with the least
                              remaining work first (each as many steps as a round allows until the time runs
                              out) */
  float long_ms;           /* TSGNE_SHARE_SHORT_FIRST: GPU time left (estimated from the measured pair rate)
                              above which a request is long (default 150) */
  float short_share;       /* TSGNE_SHARE_SHORT_FIRST: most of a round the short requests take while a long
                              one waits, in (0, 1) (default 0.3) */
} tsgne_server_config;

#define TSGNE_SHARE_EQUAL 0
#define TSGNE_SHARE_SMALLEST_FIRST 1
#define TSGNE_SHARE_SHORT_FIRST 2

typedef struct tsgne_request {
  int32_t n;             /* nodes */
  int64_t m;             /* undirected edges in edges_h */
  const int32_t* edges_h;/* int32[m][2], host; made canonical by the server (tsgne_csr_from_edges) */
  int32_t d;             /* embedding dimension */
  const float* X_h;      /* float32[n][d], host */
  const float* Y0_h;     /* float32[n][2], host */
  float perplexity;      /* > 1 */
  int32_t n_iter;        /* optimisation steps */
} tsgne_request;

typedef struct tsgne_server_stats {
  int64_t submitted, completed, failed, cancelled;
  int32_t queued, active;
  int64_t hbm_in_use, hbm_budget; /* bytes (estimated footprints) */
  int64_t rounds;
  double busy_s;                  /* time spent in rounds */
  double admit_s;                 /* worker time spent admitting requests (uploads and affinities; mostly
                                     while a round runs on the GPU) */
  double plan_s;                  /* worker time spent between rounds on plans, captures and shares */
  double latency_p50_ms, latency_p99_ms, latency_mean_ms; /* submission to completion, completed requests */
  double layouts_per_s;           /* completed / (last completion - first submission) */
} tsgne_server_stats;

TSGNE_API void tsgne_server_config_default(tsgne_server_config* c);

/* Starts a server (and its worker thread) on the current device.
 * Errors: E_INVAL (bad configuration), E_DEVICE, E_NOMEM. */
TSGNE_API tsgne_status tsgne_server_create(const tsgne_server_config* cfg, tsgne_server** out);

/* Copies the request in (making its edge list a canonical CSR on the calling
 * thread) and queues it; *ticket identifies it.  Errors: E_INVAL (bad sizes,
 * null buffers), E_NOMEM (its footprint exceeds the whole budget), E_BUSY
 * (queue full).  Graph errors (non-canonical edges are canonicalised;
 * endpoints out of range) surface as the request's result. */
TSGNE_API tsgne_status tsgne_server_submit(tsgne_server* srv, const tsgne_request* req, uint64_t* ticket);

/* Non-blocking: *done = 1 when the request has finished; then *result holds its
 * status (TSGNE_OK, E_NONFINITE, E_CANCELLED, ...) and, if TSGNE_OK and Y_h
 * is not NULL, float32[n][2] receives the layout. */
TSGNE_API tsgne_status tsgne_server_poll(tsgne_server* srv, uint64_t ticket, float* Y_h, int32_t* done,
                                         tsgne_status* result);

/* Blocks until the request has finished; outputs as tsgne_server_poll. */
TSGNE_API tsgne_status tsgne_server_wait(tsgne_server* srv, uint64_t ticket, float* Y_h, tsgne_status* result);

/* Times of a finished request that has not been released (either pointer may
 * be NULL): *latency_ms from submission to completion, *queued_ms from
 * submission to admission (to completion for a request cancelled while
 * queued).  E_INVAL for an unknown ticket, E_BUSY while queued or running. */
TSGNE_API tsgne_status tsgne_server_latency(tsgne_server* srv, uint64_t ticket, double* latency_ms, double* queued_ms);

/* The error message of a finished request that failed (empty if it
 * succeeded), copied into buf (at most len - 1 characters and a NUL).
 * E_INVAL for an unknown ticket, E_BUSY while queued or running. */
TSGNE_API tsgne_status tsgne_server_error(tsgne_server* srv, uint64_t ticket, char* buf, int32_t len);

/* Forgets a finished request (its layout copy is released).  E_BUSY if running. */
TSGNE_API tsgne_status tsgne_server_release(tsgne_server* srv, uint64_t ticket);

/* Cancels a queued request at once, an active one at the next round boundary. */
TSGNE_API tsgne_status tsgne_server_cancel(tsgne_server* srv, uint64_t ticket);

TSGNE_API tsgne_status tsgne_server_get_stats(tsgne_server* srv, tsgne_server_stats* out);

/* Stops the worker after its current round, cancels unfinished requests and
 * frees everything.  NULL is accepted. */
TSGNE_API tsgne_status tsgne_server_destroy(tsgne_server* srv);

/* ------------------------------------------------------------------------
 * One GPU's share of a row-sharded repulsion (the repulsive half of the
 * gradient of eq. (5) and Z of eq. (4)), for runs that spread one graph over
 * several GPUs.  Positions are cut into nb = ceil(n / T) blocks of T = 64 *
 * tile_rows; the symmetric tile (a, b), a <= b, holds every pair between
 * blocks a and b.  Row blocks a and nb-1-a form pair p = min(a, nb-1-a), and
 * shard s owns the tiles (a, b) whose row block a has p mod n_shards == s
 * (balanced: a pair of row blocks holds nb+1 tiles).  For its tiles a shard
 * computes, per node i,
 *   F_i = sum over pairs {i, j} of its tiles of w_ij^2 (y_i - y_j),
 *   Z_s = sum over ordered pairs (i, j), i != j, of its tiles of w_ij,
 * w_ij = (1 + ||y_i - y_j||^2)^-1, with the same tile arithmetic as the
 * single-GPU step (FP32 per pair; in TSGNE_PREC_SPLIT the cross-tile sums
 * and Z in FP64).  Summed over all shards, F_i is the repulsive sum R_i and
 * Z_s is Z, so the gradient is 4 (alpha A_i - R_i / Z) with A from
 * tsgne_attraction.  Every shard of a run must use the same n, n_shards and
 * tile_rows.
 * ------------------------------------------------------------------------ */
typedef struct tsgne_shard tsgne_shard;

/*
 * Plans shard `shard` of n_shards for n positions on the current device:
 * tile_rows 1, 2, 4, 8, 12, 14, 15 or 16, or 0 = chosen from the shard's tile
 * count.  Allocates the tile list, the partial buffer (nb * nb * T float2:
 * 8 bytes per node per block) and the Z partials; *out is library-owned,
 * release it with tsgne_shard_free.  A shard may own no tile (small n, many
 * shards); its results are then zero.  Synchronising.
 * Errors: E_INVAL (n < 1, n_shards outside [1, 65536], shard outside
 * [0, n_shards), bad tile_rows, NULL out), E_NOMEM, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_shard_create(int32_t n, int32_t shard, int32_t n_shards, int32_t tile_rows,
                                          tsgne_shard** out);

/* The shard's tile rows, tile count and ordered pairs (any may be NULL). */
TSGNE_API tsgne_status tsgne_shard_info(const tsgne_shard* sh, int32_t* tile_rows, int64_t* tiles, int64_t* pairs);

/*
 * The shard's force sums and Z partial at layout Y_d (caller-owned device
 * float32[n][2], read): F_d float64[n][2] (written for every node, zero for
 * nodes no tile of the shard touches), Z_d float64[1] (written).  precision
 * TSGNE_PREC_SPLIT or TSGNE_PREC_FP32 (FP32 sums, stored as float64).
 * Asynchronous on stream; calls on one shard must not overlap (they share its
 * partial buffer).  Errors: E_INVAL, E_DEVICE.
 */
TSGNE_API tsgne_status tsgne_shard_repulsion(tsgne_shard* sh, const float* Y_d, int32_t precision, double* F_d,
                                             double* Z_d, void* stream);

/*
 * Turns event timing of the shard's tile kernel on (enable != 0) or off and
 * clears the totals.  While on, each tsgne_shard_repulsion brackets its tile
 * kernel launch with two events on its stream.
 */
TSGNE_API tsgne_status tsgne_shard_set_timing(tsgne_shard* sh, int32_t enable);

/* Summed device time (ms) and number of timed tile-kernel launches since
 * timing was enabled (either may be NULL).  Synchronising (waits for the
 * last event). */
TSGNE_API tsgne_status tsgne_shard_timing(tsgne_shard* sh, double* tile_ms, int64_t* launches);

/* Releases a shard (waits for the device first).  NULL is accepted. */
TSGNE_API tsgne_status tsgne_shard_free(tsgne_shard* sh);

/*
 * Per-phase device timing of one graph's kernels, measured with HIP events
 * recorded on the stream each kernel is launched on.  Phases:
 */
#define TSGNE_PHASE_REPULSION 0 /* all-pairs repulsion + Z partials (one launch per step) */
#define TSGNE_PHASE_ZSUM 1      /* Z reduction */
#define TSGNE_PHASE_ATTRACT 2   /* sparse attraction */
#define TSGNE_PHASE_UPDATE 3    /* gradient combine + momentum/gains update */
#define TSGNE_PHASE_KL 4        /* KL edge sum */
#define TSGNE_NUM_PHASES 5

typedef struct tsgne_timing {
  double ms[TSGNE_NUM_PHASES];         /* summed device time per phase, milliseconds */
  int64_t launches[TSGNE_NUM_PHASES];  /* number of timed launches per phase */
} tsgne_timing;

/*
 * Turns per-phase timing of g on (enable != 0) or off and clears the totals.
 * While on, each timed launch is bracketed by two events on its stream.
 */
TSGNE_API tsgne_status tsgne_graph_set_timing(tsgne_graph* g, int32_t enable);

/* Totals since timing was enabled.  Synchronising (waits for the last event). */
TSGNE_API tsgne_status tsgne_graph_timing(tsgne_graph* g, tsgne_timing* out);

#ifdef __cplusplus
}
#endif

#endif /* TSGNE_H */
