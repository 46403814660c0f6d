"""Pins of the metric oracle (eq. knn-kl, Sec. III-F MMD) against hand-worked
values, an independent nearest-neighbour library, invariances and the
estimator's large-sample limit.  None compares the oracle with itself."""
import json
import math
import os

import numpy as np
import pytest

from oracle import metrics as om

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "metrics_hand_worked.json")


def _fixture():
    with open(GOLDEN) as f:
        return json.load(f)


def test_knn_kl_hand_worked():
    g = _fixture()["knn"]
    P = np.array(g["P"], dtype=float)[:, None]
    Q = np.array(g["Q"], dtype=float)[:, None]
    for c in g["cases"]:
        a, b = (P, Q) if c["direction"] == "P||Q" else (Q, P)
        assert abs(om.knn_kl(a, b, c["k"], c["l"]) - c["value"]) <= 1e-14, c


def test_knn_kl_dimension_factor():
    """Points on a line embedded isometrically in the plane: every distance
    is kept, so only the leading factor d changes (1 -> 2)."""
    g = _fixture()["knn"]
    s = 1.0 / math.sqrt(2.0)
    P = np.array(g["P"], dtype=float)[:, None] * np.array([[s, s]])
    Q = np.array(g["Q"], dtype=float)[:, None] * np.array([[s, s]])
    assert abs(om.knn_kl(P, Q, 1, 1) - 2 * (0.25 * math.log(0.75))) <= 1e-13


def test_mmd_hand_worked():
    g = _fixture()["mmd"]
    c = g[0]
    mm, s = om.mmd2(np.array(c["P"], float)[:, None], np.array(c["Q"], float)[:, None], sigma=c["sigma"])
    assert s == 1.0 and abs(mm - c["value"]) <= 1e-15
    c = g[1]
    mm, s = om.mmd2(np.array(c["P"], float)[:, None], np.array(c["Q"], float)[:, None])
    assert s == c["sigma_value"]
    t = 2 * s * s
    want = (math.exp(-1 / t) + math.exp(-16 / t)
            - (math.exp(-9 / t) + math.exp(-49 / t) + math.exp(-4 / t) + math.exp(-36 / t)) / 2)
    assert abs(mm - want) <= 1e-15


def test_nearest_neighbours_match_kdtree():
    """The oracle's k-th neighbour distances equal those of scipy's k-d tree
    (a different algorithm) in 7 dimensions."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(4)
    P = rng.normal(size=(60, 7))
    Q = rng.normal(size=(45, 7)) + 0.3
    k, l = 3, 2
    t = om.knn_terms(P, Q, k, l)
    nu = cKDTree(Q).query(P, k=k)[0][:, k - 1]
    rho = cKDTree(P).query(P, k=l + 1)[0][:, l]  # neighbour 0 is the point itself
    np.testing.assert_allclose(np.exp(0.5 * t[:, 0]), nu, rtol=1e-12)
    np.testing.assert_allclose(np.exp(0.5 * t[:, 1]), rho, rtol=1e-12)


def test_gram_distances_match_explicit_differences():
    """The matrix-product form used for the median of large sets agrees
    with explicit differences on trajectory-like rows."""
    from paper_2109_08815_amd import synth

    P, Q = synth.metric_sets(3, 120, 30, 900)
    Z = np.concatenate([P, Q]).astype(np.float64)
    a, b = om.sq_dists(Z, Z), om.sq_dists_gram(Z, Z)
    iu = np.triu_indices(len(Z), 1)
    np.testing.assert_allclose(b[iu], a[iu], rtol=1e-10)
    assert om.median_distance(P, Q, gram=True) == pytest.approx(om.median_distance(P, Q), rel=1e-12)


def test_invariances():
    """Distances, hence both metrics, are unchanged by a common rotation and
    translation; scaling both sets leaves KL unchanged (ratios of
    distances) and MMD unchanged with the median-heuristic bandwidth."""
    rng = np.random.default_rng(8)
    P = rng.normal(size=(40, 5))
    Q = rng.normal(size=(30, 5)) * 1.5 + 0.2
    R, _ = np.linalg.qr(rng.normal(size=(5, 5)))
    b = rng.normal(size=5)
    base = om.metrics(P, Q)
    for P2, Q2 in ((P @ R.T + b, Q @ R.T + b), (3.0 * P, 3.0 * Q)):
        got = om.metrics(P2, Q2)
        np.testing.assert_allclose(got[:3], base[:3], rtol=1e-10, atol=1e-12)


def test_weights_scale_coordinates():
    rng = np.random.default_rng(9)
    P = rng.normal(size=(20, 6))
    Q = rng.normal(size=(15, 6))
    w = rng.uniform(0.5, 2.0, 6)
    np.testing.assert_allclose(om.metrics(P, Q, w=w), om.metrics(P * w, Q * w), rtol=1e-13)


def test_knn_kl_large_sample_limit():
    """KL(N(0,1) || N(1,1)) = 1/2; the estimate from 2000 samples each lands
    near it and has the right sign in both directions (sampling error about
    0.1 at this size)."""
    rng = np.random.default_rng(1)
    P = rng.normal(0, 1, (2000, 1))
    Q = rng.normal(1, 1, (2000, 1))
    assert abs(om.knn_kl(P, Q) - 0.5) < 0.15
    assert abs(om.knn_kl(Q, P) - 0.5) < 0.15
    assert abs(om.knn_kl(P, rng.normal(0, 1, (2000, 1)))) < 0.1


def test_zero_distance_gives_infinite_term():
    """A repeated row of P makes rho = 0: the estimate diverges to +inf."""
    P = np.array([[0.0], [0.0], [1.0], [2.0], [5.0]])
    Q = np.array([[0.5], [3.0], [4.0]])
    assert om.knn_kl(P, Q, 1, 1) == math.inf


def test_argument_checks():
    P = np.zeros((3, 2))
    with pytest.raises(ValueError):
        om.knn_kl(P, P, 3, 3)
    with pytest.raises(ValueError):
        om.mmd2(P[:1], P)
