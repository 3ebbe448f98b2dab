/*
 * FP64 CPU oracle for the t-SGNE optimisation loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it, to check the HIP library against a plain, slow,
 * obviously correct implementation.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * Everything is computed in double precision from FP32 inputs promoted
 * exactly.  Each function cites the passage of the paper (Li, Xiao, Zhou,
 * "Efficiently Visualizing Large Graphs", arXiv 2310.11186) it follows; where
 * the paper is silent the reading taken is named in the comment.
 *
 * Pins: every function here is pinned by tests that do not re-type its
 * formula (finite differences, closed forms, brute force, invariants); the
 * momentum/gains update is pinned only by a hand-computed step because the
 * paper gives no optimiser.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_EGRAPH (-2)
#define ORACLE_ENOMEM (-3)

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int k) {
#ifdef _OPENMP
  if (k > 0) omp_set_num_threads(k);
#else
  (void)k;
#endif
}

/* ------------------------------------------------------------------ */
/* Graph: G = (V, E) undirected and unweighted (§2, problem statement). */
/* ------------------------------------------------------------------ */

typedef struct {
  int32_t r, c;
} pair32;

static int cmp_pair(const void* a, const void* b) {
  const pair32* x = (const pair32*)a;
  const pair32* y = (const pair32*)b;
  if (x->r != y->r) return x->r < y->r ? -1 : 1;
  if (x->c != y->c) return x->c < y->c ? -1 : 1;
  return 0;
}

/*
 * Canonical CSR of an undirected edge list (§2: G undirected, unweighted).
 * Self-loops are dropped, each edge {u,v} becomes (u,v) and (v,u), entries
 * are sorted by (row, col) and duplicates removed.  col must hold 2*m
 * entries; row_ptr n+1.  Returns ORACLE_EINVAL on an out-of-range endpoint.
 */
int oracle_csr_from_edges(int32_t n, int64_t m, const int32_t* uv, int32_t* row_ptr, int32_t* col,
                          int64_t* nnz_out) {
  if (n < 0 || m < 0) return ORACLE_EINVAL;
  pair32* e = (pair32*)malloc(sizeof(pair32) * (size_t)(2 * m + 1));
  if (!e) return ORACLE_ENOMEM;
  int64_t k = 0;
  for (int64_t t = 0; t < m; ++t) {
    int32_t u = uv[2 * t], v = uv[2 * t + 1];
    if (u < 0 || v < 0 || u >= n || v >= n) {
      free(e);
      return ORACLE_EINVAL;
    }
    if (u == v) continue;
    e[k].r = u; e[k].c = v; ++k;
    e[k].r = v; e[k].c = u; ++k;
  }
  qsort(e, (size_t)k, sizeof(pair32), cmp_pair);
  int64_t w = 0;
  for (int64_t t = 0; t < k; ++t) {
    if (w > 0 && e[t].r == e[w - 1].r && e[t].c == e[w - 1].c) continue;
    e[w++] = e[t];
  }
  for (int32_t i = 0; i <= n; ++i) row_ptr[i] = 0;
  for (int64_t t = 0; t < w; ++t) row_ptr[e[t].r + 1] += 1;
  for (int32_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
  for (int64_t t = 0; t < w; ++t) col[t] = e[t].c;
  *nnz_out = w;
  free(e);
  return ORACLE_OK;
}

static int cmp_int32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Position of column j in row i (ascending), or -1. */
static int64_t find_in_row(const int32_t* row_ptr, const int32_t* col, int32_t i, int32_t j) {
  int64_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] == j) return mid;
    if (col[mid] < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/*
 * Checks that the CSR is canonical (row_ptr monotone from 0, columns in range,
 * strictly ascending per row, no self-loops) and structurally symmetric, and
 * gives each entry e = (i, j) the position of (j, i).  The neighbourhood graph
 * of t-SGNE is built from G itself (§2.2, eq. (7)), so it inherits G's symmetry.
 */
int oracle_mirror(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, int32_t* mirror) {
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return ORACLE_EGRAPH;
  for (int32_t i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) return ORACLE_EGRAPH;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int32_t j = col[e];
      if (j < 0 || j >= n || j == i) return ORACLE_EGRAPH;
      if (e > row_ptr[i] && col[e - 1] >= j) return ORACLE_EGRAPH;
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int64_t p = find_in_row(row_ptr, col, col[e], i);
      if (p < 0) return ORACLE_EGRAPH;
      mirror[e] = (int32_t)p;
    }
  }
  return ORACLE_OK;
}

/*
 * The t-SGNE neighbourhood graph G_knn,G of §2.2, eq. (7): v_i and v_j are
 * joined when one is among the first k nearest neighbours of the other on G,
 * nearest by breadth-first search.  Reading: the first k neighbours of i are
 * the k smallest nodes j != i under (hop distance from i, node id) -- fewer
 * when i's component is smaller.  Each BFS runs level by level and stops once
 * a completed level brings the count to k.  The result is the canonical
 * symmetric CSR of the union (out_col must hold 2*n*k entries).
 */
int oracle_knn_graph(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t k, int32_t* out_row_ptr,
                     int32_t* out_col, int64_t* out_nnz) {
  if (n < 0 || k < 1) return ORACLE_EINVAL;
  int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* uv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * (int64_t)n * k + 2));
  if (!dist || !queue || !uv) {
    free(dist);
    free(queue);
    free(uv);
    return ORACLE_ENOMEM;
  }
  for (int32_t v = 0; v < n; ++v) dist[v] = -1;
  int64_t m = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t head = 0, tail = 0, taken = 0;
    queue[tail++] = i;
    dist[i] = 0;
    while (head < tail && taken < k) {
      /* expand one whole level: queue[head..level_end) */
      int32_t level_end = tail, next_begin = tail;
      for (; head < level_end; ++head) {
        int32_t u = queue[head];
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
          int32_t v = col[e];
          if (dist[v] < 0) {
            dist[v] = dist[u] + 1;
            queue[tail++] = v;
          }
        }
      }
      /* the new level, in ascending id order */
      int32_t cnt = tail - next_begin;
      qsort(queue + next_begin, (size_t)cnt, sizeof(int32_t), cmp_int32);
      for (int32_t t = next_begin; t < tail && taken < k; ++t, ++taken) {
        uv[2 * m] = i;
        uv[2 * m + 1] = queue[t];
        ++m;
      }
    }
    for (int32_t t = 0; t < tail; ++t) dist[queue[t]] = -1;
  }
  int rc = oracle_csr_from_edges(n, m, uv, out_row_ptr, out_col, out_nnz);
  free(dist);
  free(queue);
  free(uv);
  return rc;
}

/*
 * ShortestPath graph embedding (§2.3, eq. (8)): for target nodes t_0..t_{d-1},
 * E_ij = (hop distance between v_i and t_j) if it is at most l0, otherwise
 * l0 + 1 (also when no path exists).  Readings: eq. (8) writes the condition
 * on "d", read as d_ij; the prose says "less than l0" while the equation says
 * "<= l0", and the equation is followed; l0 is the real number given (the
 * paper's default is sqrt(|E|)).  One BFS from each target.  X is float32
 * [n][d] row-major.
 */
int oracle_shortest_path_embedding(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t d,
                                   const int32_t* targets, double l0, float* X) {
  if (n < 0 || d < 1) return ORACLE_EINVAL;
  int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!dist || !queue) {
    free(dist);
    free(queue);
    return ORACLE_ENOMEM;
  }
  for (int32_t j = 0; j < d; ++j) {
    int32_t t = targets[j];
    if (t < 0 || t >= n) {
      free(dist);
      free(queue);
      return ORACLE_EINVAL;
    }
    for (int32_t v = 0; v < n; ++v) dist[v] = -1;
    int32_t head = 0, tail = 0;
    queue[tail++] = t;
    dist[t] = 0;
    while (head < tail) {
      int32_t u = queue[head++];
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        int32_t v = col[e];
        if (dist[v] < 0) {
          dist[v] = dist[u] + 1;
          queue[tail++] = v;
        }
      }
    }
    for (int32_t v = 0; v < n; ++v)
      X[(int64_t)v * d + j] = (dist[v] >= 0 && (double)dist[v] <= l0) ? (float)dist[v] : (float)(l0 + 1.0);
  }
  free(dist);
  free(queue);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* Affinities P (§2.1, eqs. (2)-(3)) over graph neighbours (§2.2).      */
/* ------------------------------------------------------------------ */

/* D_e = ||x_i - x_j||^2 for each CSR entry, the squared distance of eq. (2). */
void oracle_edge_sqdist(int32_t n, const int32_t* row_ptr, const int32_t* col, const float* X, int32_t d,
                        double* D) {
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int32_t j = col[e];
      double s = 0.0;
      for (int32_t k = 0; k < d; ++k) {
        double t = (double)X[(int64_t)i * d + k] - (double)X[(int64_t)j * d + k];
        s += t * t;
      }
      D[e] = s;
    }
  }
}

/*
 * Entropy (natural log) of the row distribution p_j = exp(-beta*delta_j)/S,
 * with delta_j = D_j - D_min >= 0.  H = log S + beta * sum(delta_j e_j) / S.
 * Shifting by D_min leaves p unchanged (eq. (2) is a ratio).
 */
static double row_entropy(const double* delta, int64_t deg, double beta) {
  double S = 0.0, T = 0.0;
  for (int64_t k = 0; k < deg; ++k) {
    double ek = exp(-beta * delta[k]);
    S += ek;
    T += delta[k] * ek;
  }
  return log(S) + beta * T / S;
}

/*
 * Conditional affinities p_{j|i} of eq. (2), restricted to the graph
 * neighbours N(i) (§2.2), with 1/(2 sigma_i^2) written as beta_i and chosen by
 * binary search so that the perplexity equals perp (§2.1).
 *
 * Readings where the paper is silent:
 *  - entropy in nats with target log(perp) (equivalent to 2^H in bits);
 *  - deg_i == 0: empty row, beta_i = 0;
 *  - deg_i <= perp: the target is unreachable (max entropy is log deg_i), so
 *    the row is uniform, the beta -> 0 limit; beta_i = 0;
 *  - m = number of neighbours at the minimum distance; if m >= perp the row is
 *    uniform over those m (the beta -> infinity limit); beta_i = +inf;
 *  - otherwise the bracket starts at beta = 1/mean(delta), doubles or halves
 *    until it straddles the target, then bisects until the relative width is
 *    at most 1e-13 (or 200 halvings); beta_i is the midpoint.
 * pcond is aligned with col; beta has n entries.
 */
void oracle_calibrate(int32_t n, const int32_t* row_ptr, const double* D, double perp, double* pcond,
                      double* beta) {
  const double target = log(perp);
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    int64_t b = row_ptr[i], deg = row_ptr[i + 1] - row_ptr[i];
    if (deg == 0) {
      beta[i] = 0.0;
      continue;
    }
    if ((double)deg <= perp) {
      for (int64_t k = 0; k < deg; ++k) pcond[b + k] = 1.0 / (double)deg;
      beta[i] = 0.0;
      continue;
    }
    double dmin = D[b];
    for (int64_t k = 1; k < deg; ++k)
      if (D[b + k] < dmin) dmin = D[b + k];
    int64_t m = 0;
    for (int64_t k = 0; k < deg; ++k)
      if (D[b + k] == dmin) ++m;
    if ((double)m >= perp) {
      for (int64_t k = 0; k < deg; ++k) pcond[b + k] = (D[b + k] == dmin) ? 1.0 / (double)m : 0.0;
      beta[i] = INFINITY;
      continue;
    }
    double* delta = (double*)malloc(sizeof(double) * (size_t)(deg > 0 ? deg : 1));
    double mean = 0.0;
    for (int64_t k = 0; k < deg; ++k) {
      delta[k] = D[b + k] - dmin;
      mean += delta[k];
    }
    mean /= (double)deg;
    double b0 = 1.0 / mean, lo, hi;
    if (row_entropy(delta, deg, b0) > target) {
      lo = b0;
      hi = 2.0 * b0;
      while (row_entropy(delta, deg, hi) > target) {
        lo = hi;
        hi *= 2.0;
      }
    } else {
      hi = b0;
      lo = 0.5 * b0;
      while (row_entropy(delta, deg, lo) <= target) {
        hi = lo;
        lo *= 0.5;
      }
    }
    for (int it = 0; it < 200 && (hi - lo) > 1e-13 * hi; ++it) {
      double mid = 0.5 * (lo + hi);
      if (row_entropy(delta, deg, mid) > target) lo = mid; else hi = mid;
    }
    double bt = 0.5 * (lo + hi);
    double S = 0.0;
    for (int64_t k = 0; k < deg; ++k) S += exp(-bt * delta[k]);
    for (int64_t k = 0; k < deg; ++k) pcond[b + k] = exp(-bt * delta[k]) / S;
    beta[i] = bt;
    free(delta);
  }
}

/*
 * Joint affinities of eq. (3): p_ij = (p_{j|i} + p_{i|j}) / S on the CSR
 * pattern.  Reading: the paper's 2n assumes every row sums to one; isolated
 * nodes have empty rows, so S = 2 * (number of non-isolated nodes), which
 * makes P sum to one and equals 2n when no node is isolated.
 */
int oracle_symmetrise(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* pcond, double* P) {
  int64_t nonisolated = 0;
  for (int32_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] > row_ptr[i]) ++nonisolated;
  double S = 2.0 * (double)nonisolated;
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int64_t t = find_in_row(row_ptr, col, col[e], i);
      if (t < 0) return ORACLE_EGRAPH;
      P[e] = (pcond[e] + pcond[t]) / S;
    }
  }
  return ORACLE_OK;
}

/* Whole affinity construction: eq. (2) over N(i), perplexity search, eq. (3). */
int oracle_build_P(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const float* X, int32_t d,
                   double perp, double* P, double* beta) {
  if (perp <= 1.0 || d <= 0) return ORACLE_EINVAL;
  int32_t* mirror = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
  int rc = oracle_mirror(n, nnz, row_ptr, col, mirror);
  free(mirror);
  if (rc != ORACLE_OK) return rc;
  double* D = (double*)malloc(sizeof(double) * (size_t)(nnz + 1));
  double* pc = (double*)malloc(sizeof(double) * (size_t)(nnz + 1));
  oracle_edge_sqdist(n, row_ptr, col, X, d, D);
  oracle_calibrate(n, row_ptr, D, perp, pc, beta);
  rc = oracle_symmetrise(n, row_ptr, col, pc, P);
  free(D);
  free(pc);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Objective and gradient (§2.1, eqs. (4)-(5)).                        */
/* ------------------------------------------------------------------ */

static double kernel_w(const double* Y, int32_t i, int32_t j) {
  double dx = Y[2 * i] - Y[2 * j], dy = Y[2 * i + 1] - Y[2 * j + 1];
  return 1.0 / (1.0 + dx * dx + dy * dy);
}

/* Z = sum over ordered pairs k != l of (1 + ||y_k - y_l||^2)^-1, the
 * denominator of eq. (4).  Row sums are formed independently and added in row
 * order, so the result does not depend on the thread count. */
double oracle_Z(int32_t n, const double* Y) {
  double* rs = (double*)malloc(sizeof(double) * (size_t)(n + 1));
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t j = 0; j < n; ++j)
      if (j != i) s += kernel_w(Y, i, j);
    rs[i] = s;
  }
  double Z = 0.0;
  for (int32_t i = 0; i < n; ++i) Z += rs[i];
  free(rs);
  return Z;
}

/*
 * Gradient of eq. (5) with respect to y_i (reading: the paper states only the
 * objective; this is its analytic gradient, pinned by finite differences):
 *   g_i = 4 * sum_{j != i} (alpha * p_ij - q_ij) * w_ij * (y_i - y_j),
 * w_ij = (1 + ||y_i - y_j||^2)^-1, q_ij = w_ij / Z.  alpha is the early
 * exaggeration factor applied to P (alpha = 1 gives the plain gradient).
 * p_ij vanishes off the CSR pattern, so the attractive part runs over the
 * stored entries and the repulsive part over all j != i.
 * Rows listed in `rows` (count nrows) are computed; rows == NULL means all.
 * Z is always the full all-pairs sum.
 */
void oracle_gradient_rows(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* P, const double* Y,
                          double alpha, const int32_t* rows, int32_t nrows, double* g, double* Z_out) {
  double Z = oracle_Z(n, Y);
  int32_t count = rows ? nrows : n;
#pragma omp parallel for schedule(static)
  for (int32_t t = 0; t < count; ++t) {
    int32_t i = rows ? rows[t] : t;
    double ax = 0.0, ay = 0.0, rx = 0.0, ry = 0.0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int32_t j = col[e];
      double w = kernel_w(Y, i, j);
      ax += alpha * P[e] * w * (Y[2 * i] - Y[2 * j]);
      ay += alpha * P[e] * w * (Y[2 * i + 1] - Y[2 * j + 1]);
    }
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double w = kernel_w(Y, i, j);
      double q = w / Z;
      rx += q * w * (Y[2 * i] - Y[2 * j]);
      ry += q * w * (Y[2 * i + 1] - Y[2 * j + 1]);
    }
    g[2 * t] = 4.0 * (ax - rx);
    g[2 * t + 1] = 4.0 * (ay - ry);
  }
  if (Z_out) *Z_out = Z;
}

void oracle_gradient(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* P, const double* Y,
                     double alpha, double* g, double* Z_out) {
  oracle_gradient_rows(n, row_ptr, col, P, Y, alpha, NULL, n, g, Z_out);
}

/*
 * Repulsive sums over a subset of the pairs, to check one share of a run that
 * splits the pairs between GPUs:
 *   F_i = sum over counted j != i of w_ij^2 (y_i - y_j),
 *   Z_part = sum over counted ordered pairs (i, j), i != j, of w_ij
 * (w of eq. (4); summed over a partition of the pairs, F_i * 4 / Z is the
 * repulsive half of the gradient and Z_part adds up to Z).  The pair {i, j}
 * is counted when counted[min(group[i], group[j])] is nonzero; group == NULL
 * counts every pair.  F is written for the rows listed in `rows` (count
 * nrows; NULL = all rows, in order); Z_part only when Z_out is not NULL.
 */
static int pair_counted(const int32_t* group, const uint8_t* counted, int32_t i, int32_t j) {
  if (!group) return 1;
  int32_t gi = group[i], gj = group[j];
  return counted[gi < gj ? gi : gj] != 0;
}

void oracle_repulsion_terms(int32_t n, const double* Y, const int32_t* group, const uint8_t* counted,
                            const int32_t* rows, int32_t nrows, double* F, double* Z_out) {
  int32_t count = rows ? nrows : n;
#pragma omp parallel for schedule(static)
  for (int32_t t = 0; t < count; ++t) {
    int32_t i = rows ? rows[t] : t;
    double fx = 0.0, fy = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i || !pair_counted(group, counted, i, j)) continue;
      double w = kernel_w(Y, i, j);
      fx += w * w * (Y[2 * i] - Y[2 * j]);
      fy += w * w * (Y[2 * i + 1] - Y[2 * j + 1]);
    }
    F[2 * t] = fx;
    F[2 * t + 1] = fy;
  }
  if (!Z_out) return;
  double* rs = (double*)malloc(sizeof(double) * (size_t)(n + 1));
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    double z = 0.0;
    for (int32_t j = 0; j < n; ++j)
      if (j != i && pair_counted(group, counted, i, j)) z += kernel_w(Y, i, j);
    rs[i] = z;
  }
  double Z = 0.0;
  for (int32_t i = 0; i < n; ++i) Z += rs[i];
  free(rs);
  *Z_out = Z;
}

/* KL(P || Q) of eq. (5) with q_ij = w_ij / Z for a given Z (the all-pairs
 * sum of oracle_Z at the same Y); terms with p_ij = 0 vanish. */
double oracle_kl_given_Z(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* P, const double* Y,
                         double Z) {
  double kl = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      if (P[e] <= 0.0) continue;
      double q = kernel_w(Y, i, col[e]) / Z;
      kl += P[e] * log(P[e] / q);
    }
  }
  return kl;
}

/* KL(P || Q) of eq. (5) at Y. */
double oracle_kl(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* P, const double* Y) {
  return oracle_kl_given_Z(n, row_ptr, col, P, Y, oracle_Z(n, Y));
}

/* ------------------------------------------------------------------ */
/* Optimiser.  The paper defers it to the original t-SNE article; the  */
/* reading is gradient descent with momentum and per-coordinate gains. */
/* ------------------------------------------------------------------ */

/*
 * One update per coordinate c (reading; parity pinned only by a hand step):
 *   gain_c <- gain_c + 0.2 if g_c * u_c < 0, else 0.8 * gain_c;
 *   gain_c <- max(gain_c, min_gain);
 *   u_c    <- momentum * u_c - eta * gain_c * g_c;
 *   y_c    <- y_c + u_c.
 */
void oracle_update(int32_t n, double* Y, double* U, double* gains, const double* g, double momentum, double eta,
                   double min_gain) {
  for (int64_t c = 0; c < 2 * (int64_t)n; ++c) {
    if (g[c] * U[c] < 0.0)
      gains[c] += 0.2;
    else
      gains[c] *= 0.8;
    if (gains[c] < min_gain) gains[c] = min_gain;
    U[c] = momentum * U[c] - eta * gains[c] * g[c];
    Y[c] += U[c];
  }
}

/*
 * Steps t = t0 .. t0+n_steps-1 of the loop: exaggeration alpha = ee and
 * momentum m_early while t < t_ee, then 1 and m_late.  Y, U, gains are updated
 * in place.  If kl_trace is given, the KL at the state after each step whose
 * index+1 is a multiple of kl_every is written in order.
 */
void oracle_run(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* P, double* Y, double* U,
                double* gains, int32_t t0, int32_t n_steps, double ee, int32_t t_ee, double m_early, double m_late,
                double eta, double min_gain, int32_t kl_every, double* kl_trace) {
  double* g = (double*)malloc(sizeof(double) * (size_t)(2 * (int64_t)n + 2));
  int32_t nk = 0;
  for (int32_t t = t0; t < t0 + n_steps; ++t) {
    double alpha = t < t_ee ? ee : 1.0;
    double mom = t < t_ee ? m_early : m_late;
    oracle_gradient(n, row_ptr, col, P, Y, alpha, g, NULL);
    oracle_update(n, Y, U, gains, g, mom, eta, min_gain);
    if (kl_trace && kl_every > 0 && (t + 1) % kl_every == 0) kl_trace[nk++] = oracle_kl(n, row_ptr, col, P, Y);
  }
  free(g);
}

/* ------------------------------------------------------------------ */
/* Layout quality: NMI (section 2.5, eq. (11)) and AQ (section 2.6,     */
/* eqs. (12)-(14)).                                                      */
/* ------------------------------------------------------------------ */

/*
 * Quantised layout coordinates for the clustering of section 2.5.  Reading:
 * the paper clusters the layout with kNN clustering whose k is the number
 * of graph clusters, read as k-means (Lloyd).  So that every decision of the
 * clustering is reproducible, it runs on the layout mapped onto a 2^24 x 2^24
 * grid over its bounding box: q = min(floor((y - lo) / (hi - lo) * 2^24),
 * 2^24 - 1), 0 when hi == lo.  Returns ORACLE_EINVAL on a non-finite
 * coordinate.
 */
static int quantise_layout(int32_t n, const float* Y, int32_t* q) {
  for (int a = 0; a < 2; ++a) {
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t i = 0; i < n; ++i) {
      const double v = (double)Y[2 * (int64_t)i + a];
      if (!isfinite(v)) return ORACLE_EINVAL;
      if (v < lo) lo = v;
      if (v > hi) hi = v;
    }
    const double span = hi - lo;
    for (int32_t i = 0; i < n; ++i) {
      int32_t u = 0;
      if (span > 0) {
        const double t = floor(((double)Y[2 * (int64_t)i + a] - lo) / span * 16777216.0);
        u = t > 16777215.0 ? 16777215 : (int32_t)t;
      }
      q[2 * (int64_t)i + a] = u;
    }
  }
  return ORACLE_OK;
}

/*
 * k-means (Lloyd) on the quantised layout, the clustering of the layout in
 * section 2.5.  Readings: the initial centres are the points at the k given
 * node indices (the caller draws them); each pass assigns every point to the
 * nearest centre by squared Euclidean distance in FP64 (ties to the lower
 * cluster index), stops when no label changes, and otherwise moves every
 * non-empty cluster's centre to the mean of its points (exact integer sums,
 * one division); an empty cluster keeps its centre.  At most max_iter
 * passes; *iters receives the number made.
 */
int oracle_kmeans(int32_t n, const float* Y, int32_t k, const int32_t* seeds, int32_t max_iter, int32_t* labels,
                  int32_t* iters) {
  if (n < 1 || k < 1 || max_iter < 1) return ORACLE_EINVAL;
  int32_t* q = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n);
  double* cx = (double*)malloc(sizeof(double) * (size_t)k);
  double* cy = (double*)malloc(sizeof(double) * (size_t)k);
  int64_t* sx = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int64_t* sy = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int rc = ORACLE_OK;
  if (!q || !cx || !cy || !sx || !sy || !cnt) {
    rc = ORACLE_ENOMEM;
    goto done;
  }
  rc = quantise_layout(n, Y, q);
  if (rc != ORACLE_OK) goto done;
  for (int32_t c = 0; c < k; ++c) {
    if (seeds[c] < 0 || seeds[c] >= n) {
      rc = ORACLE_EINVAL;
      goto done;
    }
    cx[c] = (double)q[2 * (int64_t)seeds[c]];
    cy[c] = (double)q[2 * (int64_t)seeds[c] + 1];
  }
  for (int32_t i = 0; i < n; ++i) labels[i] = -1;
  int32_t it = 0;
  while (it < max_iter) {
    ++it;
    int64_t changed = 0;
    for (int32_t i = 0; i < n; ++i) {
      const double px = (double)q[2 * (int64_t)i], py = (double)q[2 * (int64_t)i + 1];
      int32_t best = 0;
      double bd = INFINITY;
      for (int32_t c = 0; c < k; ++c) {
        const double dx = px - cx[c], dy = py - cy[c];
        const double dist = dx * dx + dy * dy;
        if (dist < bd) {
          bd = dist;
          best = c;
        }
      }
      if (labels[i] != best) ++changed;
      labels[i] = best;
    }
    if (changed == 0) break;
    for (int32_t c = 0; c < k; ++c) sx[c] = sy[c] = cnt[c] = 0;
    for (int32_t i = 0; i < n; ++i) {
      sx[labels[i]] += q[2 * (int64_t)i];
      sy[labels[i]] += q[2 * (int64_t)i + 1];
      cnt[labels[i]] += 1;
    }
    for (int32_t c = 0; c < k; ++c) {
      if (cnt[c] > 0) {
        cx[c] = (double)sx[c] / (double)cnt[c];
        cy[c] = (double)sy[c] / (double)cnt[c];
      }
    }
  }
  *iters = it;
done:
  free(q);
  free(cx);
  free(cy);
  free(sx);
  free(sy);
  free(cnt);
  return rc;
}

/*
 * NMI of two labelings (section 2.5, eq. (11)): 2 I(A;B) / (H(A) + H(B)) with
 * natural logarithms (the base cancels).  Readings: the paper's remark that a
 * smaller NMI means more similar partitions is reversed in its own formula
 * (identical partitions give 1); when both labelings have a single cluster,
 * H(A) + H(B) = 0 and the NMI is taken as 1.  Labels lie in [0, ka) and
 * [0, kb).  Returns NaN on a label out of range.
 */
double oracle_nmi(int32_t n, const int32_t* a, int32_t ka, const int32_t* b, int32_t kb) {
  if (n < 1 || ka < 1 || kb < 1) return NAN;
  int64_t* nij = (int64_t*)calloc((size_t)ka * (size_t)kb, sizeof(int64_t));
  int64_t* na = (int64_t*)calloc((size_t)ka, sizeof(int64_t));
  int64_t* nb = (int64_t*)calloc((size_t)kb, sizeof(int64_t));
  double result = NAN;
  if (!nij || !na || !nb) goto done;
  for (int32_t i = 0; i < n; ++i) {
    if (a[i] < 0 || a[i] >= ka || b[i] < 0 || b[i] >= kb) goto done;
    nij[(int64_t)a[i] * kb + b[i]] += 1;
    na[a[i]] += 1;
    nb[b[i]] += 1;
  }
  {
    const double N = (double)n;
    double ha = 0, hb = 0, mi = 0;
    for (int32_t x = 0; x < ka; ++x)
      if (na[x] > 0) ha -= ((double)na[x] / N) * log((double)na[x] / N);
    for (int32_t y = 0; y < kb; ++y)
      if (nb[y] > 0) hb -= ((double)nb[y] / N) * log((double)nb[y] / N);
    for (int32_t x = 0; x < ka; ++x)
      for (int32_t y = 0; y < kb; ++y) {
        const int64_t c = nij[(int64_t)x * kb + y];
        if (c > 0) mi += ((double)c / N) * log(N * (double)c / ((double)na[x] * (double)nb[y]));
      }
    result = (ha + hb > 0) ? 2.0 * mi / (ha + hb) : 1.0;
  }
done:
  free(nij);
  free(na);
  free(nb);
  return result;
}

/*
 * Aesthetic quality (section 2.6, eqs. (12)-(14)): the layout's bounding box
 * is cut into grid x grid cells of width x0 = (Xmax - Xmin) / grid and height
 * y0 = (Ymax - Ymin) / grid; a cell is good when the largest fraction of its
 * points that share one cluster label exceeds p; AQ = good cells / grid^2.
 * Readings: a point on the upper edge belongs to the last cell; an empty cell
 * is not good; a degenerate axis (max == min) puts every point in its first
 * cell.  Returns NaN on a non-finite coordinate or a label out of range.
 */
double oracle_aq(int32_t n, const float* Y, const int32_t* labels, int32_t n_labels, int32_t grid, double p) {
  if (n < 1 || n_labels < 1 || grid < 1) return NAN;
  double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
  for (int32_t i = 0; i < n; ++i)
    for (int a = 0; a < 2; ++a) {
      const double v = (double)Y[2 * (int64_t)i + a];
      if (!isfinite(v)) return NAN;
      if (v < lo[a]) lo[a] = v;
      if (v > hi[a]) hi[a] = v;
    }
  const double w[2] = {(hi[0] - lo[0]) / grid, (hi[1] - lo[1]) / grid};
  const int64_t cells = (int64_t)grid * grid;
  int64_t* count = (int64_t*)calloc((size_t)cells * (size_t)n_labels, sizeof(int64_t));
  if (!count) return NAN;
  double result = NAN;
  for (int32_t i = 0; i < n; ++i) {
    if (labels[i] < 0 || labels[i] >= n_labels) goto done;
    int64_t cell[2];
    for (int a = 0; a < 2; ++a) {
      int64_t c = 0;
      if (w[a] > 0) {
        const double t = floor(((double)Y[2 * (int64_t)i + a] - lo[a]) / w[a]);
        c = t > grid - 1 ? grid - 1 : (int64_t)t;
      }
      cell[a] = c;
    }
    count[(cell[1] * grid + cell[0]) * n_labels + labels[i]] += 1;
  }
  {
    int64_t good = 0;
    for (int64_t c = 0; c < cells; ++c) {
      int64_t total = 0, best = 0;
      for (int32_t l = 0; l < n_labels; ++l) {
        const int64_t v = count[c * n_labels + l];
        total += v;
        if (v > best) best = v;
      }
      if (total > 0 && (double)best / (double)total > p) ++good;
    }
    result = (double)good / (double)cells;
  }
done:
  free(count);
  return result;
}

/* ------------------------------------------------------------------ */
/* Random-walk P (section 2.1, the approximation of P by random walks). */
/* ------------------------------------------------------------------ */

/*
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds of the 4x32 Philox S-box with
 * multipliers 0xD2511F53 and 0xCD9E8D57, the key advanced by the Weyl
 * constants 0x9E3779B9 and 0xBB67AE85 between rounds.
 */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c[0];
  out[1] = c[1];
  out[2] = c[2];
  out[3] = c[3];
}

/* The uniform draw of step s of walk w from node i: 53 bits of Philox output
 * for counter (i, w, s, 0) and the 64-bit seed as key, in [0, 1). */
static double walk_uniform(uint64_t seed, int32_t i, int32_t w, int32_t s) {
  const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)w, (uint32_t)s, 0u};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  oracle_philox4x32_10(ctr, key, x);
  return ((double)x[0] * 2097152.0 + (double)(x[1] >> 11)) * 0x1p-53;
}

static int cmp_u64(const void* a, const void* b) {
  const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

/*
 * P from random walks (section 2.1).  Readings: walks run on the given graph
 * (its CSR, canonical and symmetric); from node u the next node is the
 * neighbour v with probability proportional to exp(-||x_u - x_v||^2) (the
 * printed exponent lacks its minus sign), evaluated as exp(-(D_uv - D_min,u))
 * with D summed over the coordinates in order in FP64; the neighbour is the
 * first CSR entry whose running weight sum exceeds u * (row total), u the
 * uniform of walk_uniform (the last entry if none does).  Each node starts
 * `walks` walks of `length` steps (a walk from an isolated node stays put);
 * p_{j|i} = (walks from i ending at j != i) / walks, and symmetrising as in
 * eq. (3) with S the total mass gives P_ij = (c_ij + c_ji) / (2 M), M the
 * walks that do not end where they started.  The support (pairs with
 * c_ij + c_ji > 0) is returned as a canonical symmetric CSR with P aligned
 * with col; out_col and P need room for 2 n walks entries.
 */
int oracle_walk_P(int32_t n, const int32_t* row_ptr, const int32_t* col, const float* X, int32_t d, int32_t walks,
                  int32_t length, uint64_t seed, int32_t* out_row_ptr, int32_t* out_col, float* P, int64_t* out_nnz) {
  if (n < 1 || d < 1 || walks < 1 || length < 1) return ORACLE_EINVAL;
  const int64_t nnz = row_ptr[n];
  double* C = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * 2 * (size_t)n * (size_t)walks);
  if (!C || !keys) {
    free(C);
    free(keys);
    return ORACLE_ENOMEM;
  }
  /* running transition weights per row */
  for (int32_t u = 0; u < n; ++u) {
    double dmin = INFINITY;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      double D = 0;
      for (int32_t k = 0; k < d; ++k) {
        const double t = (double)X[(int64_t)u * d + k] - (double)X[(int64_t)col[e] * d + k];
        D += t * t;
      }
      C[e] = D;
      if (D < dmin) dmin = D;
    }
    double run = 0;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      run += exp(-(C[e] - dmin));
      C[e] = run;
    }
  }
  int64_t m = 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t w = 0; w < walks; ++w) {
      int32_t u = i;
      for (int32_t s = 0; s < length; ++s) {
        const int64_t a = row_ptr[u], b = row_ptr[u + 1];
        if (a == b) break;
        const double r = walk_uniform(seed, i, w, s) * C[b - 1];
        int64_t pick = b - 1;
        for (int64_t e = a; e < b; ++e)
          if (C[e] > r) {
            pick = e;
            break;
          }
        u = col[pick];
      }
      if (u != i) {
        keys[m++] = ((uint64_t)(uint32_t)i << 32) | (uint32_t)u;
        keys[m++] = ((uint64_t)(uint32_t)u << 32) | (uint32_t)i;
      }
    }
  }
  qsort(keys, (size_t)m, sizeof(uint64_t), cmp_u64);
  int64_t out = 0;
  for (int32_t r = 0; r <= n; ++r) out_row_ptr[r] = 0;
  for (int64_t a = 0; a < m;) {
    int64_t b = a;
    while (b < m && keys[b] == keys[a]) ++b;
    const int32_t row = (int32_t)(keys[a] >> 32);
    out_col[out] = (int32_t)(keys[a] & 0xffffffffu);
    P[out] = (float)((double)(b - a) / (double)m); /* (c_ij + c_ji) / (2 M), m = 2 M */
    out_row_ptr[row + 1] += 1;
    ++out;
    a = b;
  }
  for (int32_t r = 0; r < n; ++r) out_row_ptr[r + 1] += out_row_ptr[r];
  *out_nnz = out;
  free(C);
  free(keys);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* Locality order of the nodes by their embedding.                     */
/* ------------------------------------------------------------------ */

typedef struct {
  uint64_t key;
  int32_t id;
} keyed_node;

static int cmp_keyed(const void* a, const void* b) {
  const keyed_node* x = (const keyed_node*)a;
  const keyed_node* y = (const keyed_node*)b;
  if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
  return (x->id > y->id) - (x->id < y->id);
}

/*
 * A node order along a space-filling curve of the embedding.  The premise of
 * t-SGNE (section 2.2) is that nodes close in the graph are close in R^d, so
 * numbering the nodes in this order puts most graph neighbours at nearby
 * ids.  Definition: m = min(d, 8) leading coordinates, b = 64 / m bits each;
 * coordinate c of node i is quantised over its own range as
 * q = min(floor((x - lo) / (hi - lo) * 2^b), 2^b - 1) (0 on a flat axis); the
 * key is the Morton code that takes bit t of q_0, ..., q_{m-1} (in that
 * order) for t = b - 1 down to 0, most significant first.  perm[r] is the
 * node of rank r under (key, node id).
 */
int oracle_locality_order(int32_t n, const float* X, int32_t d, int32_t* perm) {
  if (n < 1 || d < 1) return ORACLE_EINVAL;
  const int m = d < 8 ? d : 8;
  const int b = 64 / m;
  keyed_node* kn = (keyed_node*)calloc((size_t)n, sizeof(keyed_node));
  uint64_t* q = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n * m);
  if (!kn || !q) {
    free(kn);
    free(q);
    return ORACLE_ENOMEM;
  }
  const double scale = ldexp(1.0, b);
  const uint64_t top = (b == 64) ? ~0ull : ((1ull << b) - 1);
  for (int c = 0; c < m; ++c) {
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t i = 0; i < n; ++i) {
      const double v = (double)X[(int64_t)i * d + c];
      if (!isfinite(v)) {
        free(kn);
        free(q);
        return ORACLE_EINVAL;
      }
      if (v < lo) lo = v;
      if (v > hi) hi = v;
    }
    const double span = hi - lo;
    for (int32_t i = 0; i < n; ++i) {
      uint64_t u = 0;
      if (span > 0) {
        const double t = floor(((double)X[(int64_t)i * d + c] - lo) / span * scale);
        u = t >= (double)top ? top : (uint64_t)t;
      }
      q[(int64_t)i * m + c] = u;
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    uint64_t key = 0;
    for (int t = b - 1; t >= 0; --t)
      for (int c = 0; c < m; ++c) key = (key << 1) | ((q[(int64_t)i * m + c] >> t) & 1u);
    kn[i].key = key;
    kn[i].id = i;
  }
  qsort(kn, (size_t)n, sizeof(keyed_node), cmp_keyed);
  for (int32_t r = 0; r < n; ++r) perm[r] = kn[r].id;
  free(kn);
  free(q);
  return ORACLE_OK;
}
