"""Parity bars shared by the GPU tests, and the per-row gradient check.

Bars (FP32 pair arithmetic with FP64 reductions, the default precision split):

* gradient: relative L2 <= GRAD_TOL of the FP64 gradient at the same Y
  (eqs. (4)-(5)); and row by row, |g_i - g64_i| <= ROW_TOL * (|4 alpha A_i| +
  |4 R_i / Z|), the sizes of the two terms the row's gradient is the
  difference of (A_i = sum_j p_ij w_ij (y_i - y_j), R_i = sum_j w_ij^2 (y_i -
  y_j)), so that a wrong row with a small force cannot hide under the norm.
* Z: |Z / Z64 - 1| <= Z_TOL.  Each pair weight w_ij is formed in FP32 (one
  rounding of 1 + d^2 and a reciprocal within 1 ulp), so Z carries errors of a
  few 1e-8 of a single weight that average out only partly over the pairs;
  measured at most 8.3e-9 over every tile size, variant and state the tests
  use.  A bar of 1e-9 would need FP64 pair weights.
* KL: |KL - KL64| <= KL_TOL * max(1, |KL64|).  P is stored in FP32 (computed
  in FP64): each stored entry carries a relative rounding of up to 2^-24, and
  KL moves by at most 2^-24 * sum_e P_e |log(P_e / q_e) + 1| ~ 6e-8 (KL + 1)
  from it; Z adds its own relative error (Z_TOL).  On small graphs whose rows
  are uniform the roundings repeat and do not average out (a 900-node SBM:
  sum of the stored P = 1 + 1.9e-8, KL moved by 2.3e-8 of KL); measured at
  most 2.3e-8 of KL, against 1.3e-9 to 3e-9 on 3,000-300,000-node graphs.
"""
import numpy as np

import oracle

GRAD_TOL = 1e-5
ROW_TOL = 1e-5
Z_TOL = 3e-8
KL_TOL = 1e-7
P_TOL = 1e-6


def kl_close(kl, kl64):
    """The KL bar: |kl - kl64| <= KL_TOL * max(1, |kl64|)."""
    return abs(kl - kl64) <= KL_TOL * max(1.0, abs(kl64))


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def row_error_ratio(g, og, Y, Z, rows=None):
    """max over rows of |g_i - og_i| / (|4 alpha A_i| + |4 R_i / Z|), and the
    row (index into `rows` when given) where it occurs.

    g, og: the rows' gradients (GPU, oracle FP64); Y: the whole layout; Z the
    oracle's normaliser at Y.  R_i comes from the oracle's repulsive sums and
    4 alpha A_i = og_i + 4 R_i / Z (the gradient is their difference)."""
    F, _ = oracle.repulsion_terms(np.asarray(Y, np.float64), rows=rows, with_Z=False)
    rep = 4.0 * F / Z
    att = np.asarray(og, np.float64) + rep
    scale = np.linalg.norm(att, axis=1) + np.linalg.norm(rep, axis=1)
    err = np.linalg.norm(np.asarray(g, np.float64) - og, axis=1)
    ratio = err / np.maximum(scale, 1e-300)
    k = int(np.argmax(ratio)) if ratio.size else 0
    return (float(ratio[k]) if ratio.size else 0.0), k


def sample_rows(n, count, seed, tile_rows=(1, 2, 4, 8, 12, 14, 15, 16)):
    """`count` seeded random rows plus the first and last row and the first
    row of the last (possibly partial) block of every tile length 64 * R."""
    rng = np.random.default_rng(seed)
    rows = set(rng.choice(n, min(count, n), replace=False).tolist())
    rows.update({0, n - 1})
    for R in tile_rows:
        T = 64 * R
        rows.add(((n - 1) // T) * T)
    return np.array(sorted(rows), np.int32)
