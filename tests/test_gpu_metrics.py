"""Parity of the GPU consistency metrics (pds_traj_metrics, through the C
ABI) with the FP64 oracle on the same float32 rows.

Tolerances follow from the GPU's arithmetic: a squared distance is a sum of
FP32 squared differences over chunks of 32 coordinates, added in FP64, so
its relative error is at most about 33 * 2^-24 < EPS = 2.5e-6.  Then
* KL: each row adds d/2 (log nu^2 - log rho^2); nu^2 and rho^2 are order
  statistics of values each within EPS relative, so each log moves by at
  most EPS and the estimate by at most d EPS;
* sigma: the square root of (a mean of) order statistics: EPS / 2 relative
  (the median's ranks are selected exactly on the GPU's own values);
* MMD^2: a kernel value exp(-x) with x = d^2 / (2 sigma^2) moves by at most
  x e^-x (EPS + 2 EPS / 2) <= 2 EPS / e, and MMD^2 combines four means of
  them (weights 1, 1, 2): 8 EPS / e.
"""
import math

import numpy as np
import pytest
import torch

from oracle import metrics as om
from paper_2109_08815_amd import lib as L
from paper_2109_08815_amd import synth
from tests.helpers import print_case, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

EPS = 2.5e-6


def gpu_metrics(P, Q, w=None, k=3, l=3, sigma=None, rows=False):
    dev = torch.device("cuda")
    Pt = torch.as_tensor(P, device=dev)
    Qt = torch.as_tensor(Q, device=dev)
    wt = torch.as_tensor(np.asarray(w, dtype=np.float32), device=dev) if w is not None else None
    r = L.traj_metrics(Pt, Qt, wt, k, l, sigma, rows=rows)
    torch.cuda.synchronize()
    if rows:
        return r[0].cpu().numpy(), r[1].cpu().numpy()
    return r.cpu().numpy()


def check(P, Q, w=None, k=3, l=3, sigma=None):
    d = P.shape[1]
    got = gpu_metrics(P, Q, w, k, l, sigma)
    ref = om.metrics(P.astype(np.float64), Q.astype(np.float64), k, l, sigma,
                     None if w is None else np.asarray(w, np.float32).astype(np.float64))
    for i in (0, 1):
        assert abs(got[i] - ref[i]) <= d * EPS + 1e-12 * abs(ref[i]), (i, got[i], ref[i])
    assert abs(got[3] - ref[3]) <= 0.5 * EPS * ref[3] + 1e-300, (got[3], ref[3])
    assert abs(got[2] - ref[2]) <= 8 * EPS / math.e + 1e-12, (got[2], ref[2])
    return got, ref


CASES = [
    ("ragged, split coordinates", dict(n=150, m=37, d=203)),
    ("one split, diagonal tiles", dict(n=300, m=60, d=30)),
    ("many tiles", dict(n=1500, m=200, d=40)),
    ("smallest sets", dict(n=4, m=4, d=1)),
    ("k 2, l 5", dict(n=40, m=30, d=100, k=2, l=5)),
    ("given sigma", dict(n=60, m=25, d=50, sigma=2.5)),
    ("spread posterior", dict(n=200, m=10, d=400, spread=3.0)),
]


@pytest.mark.parametrize("name,c", CASES)
def test_metrics_match_oracle(name, c):
    print_case("metrics", name, c)
    c = dict(c)
    P, Q = synth.metric_sets(11, c.pop("n"), c.pop("m"), c.pop("d"), spread=c.pop("spread", 1.0))
    check(P, Q, **c)


def test_metrics_with_weights():
    print_case("metrics weights")
    P, Q = synth.metric_sets(12, 70, 20, 64)
    w = np.random.default_rng(3).uniform(0.5, 100.0, 64).astype(np.float32)
    check(P, Q, w=w)


def test_repeated_row_gives_infinite_estimate():
    """With k = l = 1, rho = 0 for a repeated row of P: KL(P||Q) is +inf on
    both sides, KL(Q||P) stays finite."""
    print_case("metrics repeated row")
    P, Q = synth.metric_sets(13, 20, 12, 16)
    P[1] = P[0]
    got = gpu_metrics(P, Q, k=1, l=1)
    ref = om.metrics(P.astype(np.float64), Q.astype(np.float64), 1, 1)
    assert got[0] == math.inf and ref[0] == math.inf
    assert np.isfinite(got[1]) and abs(got[1] - ref[1]) <= 16 * EPS + 1e-12 * abs(ref[1])


def test_repeatable_bitwise():
    print_case("metrics repeat")
    P, Q = synth.metric_sets(14, 300, 40, 128)
    a = gpu_metrics(P, Q)
    b = gpu_metrics(P, Q)
    np.testing.assert_array_equal(a, b)


@pytest.mark.slow
def test_full_size_rollout_sets_sampled():
    """The benchmark's size (1024 rollouts of 1000 steps x 5 joint angles
    against 10 held-out trajectories): sigma against the oracle's median
    over all pairs, the per-row terms of a row sample against the oracle's
    explicit differences, and the four outputs against fixed-order sums of
    the GPU's own rows."""
    print_case("metrics full size")
    n, m, d = 1024, 10, 5000
    P, Q = synth.metric_sets(15, n, m, d)
    out, rows = gpu_metrics(P, Q, rows=True)
    sig = om.median_distance(P, Q, gram=True)
    assert abs(out[3] - sig) <= 0.5 * EPS * sig
    Z = np.concatenate([P, Q]).astype(np.float64)
    sel = np.array([0, 1, 63, 64, 511, 1000, 1023, 1024, 1029, 1033])
    ref = om.row_terms(Z, n, 3, 3, sig, sel)
    assert np.all(np.abs(rows[sel, 0] - ref[:, 0]) <= d * EPS)
    assert np.all(np.abs(rows[sel, 1:] - ref[:, 1:]) <= (n + m) * 2 * EPS / math.e)
    # outputs from the rows
    dpsi = 0.0
    kl_pq = rows[:n, 0].sum() / n + dpsi + math.log(m / (n - 1))
    kl_qp = rows[n:, 0].sum() / m + dpsi + math.log(n / (m - 1))
    mmd = rows[:n, 1].sum() / (n * (n - 1)) + rows[n:, 1].sum() / (m * (m - 1)) - 2 * rows[:n, 2].sum() / (n * m)
    np.testing.assert_allclose(out[:3], [kl_pq, kl_qp, mmd], rtol=1e-12, atol=1e-12)
    # the cross sums seen from both sides agree
    assert abs(rows[:n, 2].sum() - rows[n:, 2].sum()) <= 1e-9 * rows[:n, 2].sum()
