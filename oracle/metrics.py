"""FP64 CPU oracle of the posterior-consistency metrics (Sec. III-F, App. A-D).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the CPU-baseline
leg of the benchmark, never by the GPU library or its Python binding.  It
shares no code with the HIP path.

What is computed, for two sets of trajectories given as rows (each row one
trajectory's observations, flattened to d numbers):

* ``knn_kl(P, Q, k, l)``: the k-nearest-neighbour KL estimate of eq.
  knn-kl (after Wang et al.),
      d/n sum_i log(nu_k(i) / rho_l(i)) + psi(l) - psi(k) + log(m / (n - 1)),
  with n = |P|, m = |Q|, nu_k(i) the Euclidean distance from P_i to its k-th
  nearest row of Q, rho_l(i) the distance from P_i to its l-th nearest row
  of P without P_i, d the row length.  The paper takes k = l = 3.
* ``mmd2(P, Q, sigma)``: the squared maximum mean discrepancy of Sec. III-F
  (Gretton et al.), as the unbiased U-statistic
      1/(n(n-1)) sum_{i!=j} k(P_i,P_j) + 1/(m(m-1)) sum_{i!=j} k(Q_i,Q_j)
      - 2/(nm) sum_{i,j} k(P_i,Q_j).
  The paper names no kernel; this reading takes the Gaussian kernel
  k(x, y) = exp(-||x - y||^2 / (2 sigma^2)) with sigma the median distance
  over all distinct pairs of the pooled set P u Q (median heuristic; the
  mean of the two middle distances for an even count), sigma = 1 when that
  median is 0.
* ``row_terms``: the per-row quantities both sums are made of, for checks at
  sizes where the full oracle would be slow.

Distances are explicit differences, squared and summed in FP64 (for the
median of very large sets optionally norms plus an FP64 matrix product);
the nearest neighbours come from a full sort of each row.  Optional per-column
weights w scale each coordinate before the distances (w = 1 / sigma_obs
turns observations into standardised residual space).
"""
from __future__ import annotations

import math

import numpy as np


def _rows(X, w):
    X = np.asarray(X, dtype=np.float64)
    if X.ndim != 2:
        raise ValueError("trajectory sets are [rows, d] arrays")
    if w is not None:
        X = X * np.asarray(w, dtype=np.float64)[None, :]
    return X


def sq_dists(X, Y):
    """[|X|, |Y|] squared Euclidean distances, row by row from explicit
    differences (no expansion into norms and dot products)."""
    out = np.empty((X.shape[0], Y.shape[0]))
    for i in range(X.shape[0]):
        diff = Y - X[i][None, :]
        out[i] = (diff * diff).sum(axis=1)
    return out


def harmonic(n: int) -> float:
    """H_n = 1 + 1/2 + ... + 1/n (H_0 = 0); psi(b) - psi(a) = H_{b-1} - H_{a-1}
    for positive integers a, b."""
    return sum(1.0 / j for j in range(1, n + 1))


def _kth(sorted_row, k):
    return sorted_row[k - 1]


def knn_terms(P, Q, k, l, w=None):
    """Per row of P: (log nu_k^2, log rho_l^2), from squared distances."""
    P, Q = _rows(P, w), _rows(Q, w)
    n = P.shape[0]
    dpq = sq_dists(P, Q)
    dpp = sq_dists(P, P)
    out = np.empty((n, 2))
    with np.errstate(divide="ignore"):
        for i in range(n):
            nu2 = _kth(np.sort(dpq[i]), k)
            rho2 = _kth(np.sort(np.delete(dpp[i], i)), l)
            out[i] = (math.log(nu2) if nu2 > 0 else -math.inf, math.log(rho2) if rho2 > 0 else -math.inf)
    return out


def knn_kl(P, Q, k=3, l=3, w=None):
    """Eq. knn-kl: estimate of d_KL(P || Q) from samples (rows)."""
    n, m, d = len(P), len(Q), np.asarray(P).shape[1]
    if n < l + 1 or m < k or k < 1 or l < 1:
        raise ValueError("need |P| >= l + 1 and |Q| >= k")
    t = knn_terms(P, Q, k, l, w)
    with np.errstate(invalid="ignore"):
        s = float(np.sum(0.5 * d * (t[:, 0] - t[:, 1])))
    return s / n + (harmonic(l - 1) - harmonic(k - 1)) + math.log(m / (n - 1))


def sq_dists_gram(X, Y):
    """The same squared distances as ||x||^2 + ||y||^2 - 2 x.y with an FP64
    matrix product (for sets too large for explicit differences; the FP64
    cancellation stays far below the GPU's FP32 tolerance)."""
    nx = (X * X).sum(axis=1)
    ny = (Y * Y).sum(axis=1)
    return np.maximum(nx[:, None] + ny[None, :] - 2.0 * (X @ Y.T), 0.0)


def median_distance(P, Q, w=None, gram=False):
    """Median of the Euclidean distances over all distinct pairs of P u Q."""
    Z = np.concatenate([_rows(P, w), _rows(Q, w)])
    D2 = sq_dists_gram(Z, Z) if gram else sq_dists(Z, Z)
    iu = np.triu_indices(Z.shape[0], 1)
    return float(np.median(np.sqrt(D2[iu])))


def mmd2(P, Q, sigma=None, w=None):
    """Unbiased squared MMD with the Gaussian kernel (see module docstring)."""
    Pw, Qw = _rows(P, w), _rows(Q, w)
    n, m = Pw.shape[0], Qw.shape[0]
    if n < 2 or m < 2:
        raise ValueError("MMD needs two rows in each set")
    if sigma is None:
        sigma = median_distance(P, Q, w)
        if sigma * sigma < 1e-300:
            sigma = 1.0
    g = 1.0 / (2.0 * sigma * sigma)
    kpp = np.exp(-sq_dists(Pw, Pw) * g)
    kqq = np.exp(-sq_dists(Qw, Qw) * g)
    kpq = np.exp(-sq_dists(Pw, Qw) * g)
    spp = kpp.sum() - np.trace(kpp)
    sqq = kqq.sum() - np.trace(kqq)
    return float(spp / (n * (n - 1)) + sqq / (m * (m - 1)) - 2.0 * kpq.sum() / (n * m)), float(sigma)


def metrics(P, Q, k=3, l=3, sigma=None, w=None):
    """(KL(P||Q), KL(Q||P), MMD^2, sigma) — the four numbers the GPU entry
    point returns."""
    mm, s = mmd2(P, Q, sigma, w)
    return knn_kl(P, Q, k, l, w), knn_kl(Q, P, k, l, w), mm, s


def row_terms(Z_rows, n, k, l, sigma, sel, w=None):
    """For selected rows r of the pooled set Z = P u Q (first n rows are P):
    (0.5 d (log nu_k^2 - log rho_l^2), sum_{j in own set, j != r} k_rj,
    sum_{j in the other set} k_rj), with nu taken over the other set and
    rho over the own set without r."""
    Z = _rows(Z_rows, w)
    R, d = Z.shape
    g = 1.0 / (2.0 * sigma * sigma)
    out = np.empty((len(sel), 3))
    for a, r in enumerate(sel):
        d2 = sq_dists(Z[r:r + 1], Z)[0]
        own = np.arange(R) < n if r < n else np.arange(R) >= n
        own_d = np.delete(d2, r)[np.delete(own, r)]
        oth_d = d2[~own]
        with np.errstate(divide="ignore", invalid="ignore"):
            nu2, rho2 = np.sort(oth_d)[k - 1], np.sort(own_d)[l - 1]
            out[a, 0] = 0.5 * d * (np.log(nu2) - np.log(rho2))
        out[a, 1] = np.exp(-own_d * g).sum()
        out[a, 2] = np.exp(-oth_d * g).sum()
    return out
