"""Pins of the FP64 streaming K-means oracle (Eq. 10): scikit-learn's Lloyd
iteration, closed forms, brute force over partitions and invariants."""
import itertools

import numpy as np
import pytest

from oracle import kmeans_oracle as KM


def _blobs(rng, k, per, D, spread=0.05, scale=1.0):
    centres = scale * rng.standard_normal((k, D))
    X = np.repeat(centres, per, axis=0) + spread * rng.standard_normal((k * per, D))
    return X, centres


def test_sqdist_matches_expanded_form():
    rng = np.random.default_rng(0)
    X, C = rng.standard_normal((50, 7)), rng.standard_normal((9, 7))
    ref = (X ** 2).sum(1)[:, None] - 2 * X @ C.T + (C ** 2).sum(1)[None, :]
    np.testing.assert_allclose(KM.sqdist(X, C), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("weighted", [False, True])
def test_lloyd_matches_sklearn(weighted):
    sk = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(1)
    X = rng.standard_normal((400, 12))
    w = rng.uniform(0.2, 3.0, 400) if weighted else None
    C0 = X[rng.choice(400, 10, replace=False)]
    for iters in (1, 3, 8):
        C, W, a = KM.lloyd(X, w, C0, iters)
        assert np.all(W > 0)  # no empty cluster: sklearn would relocate one
        ref = sk.KMeans(n_clusters=10, init=C0, n_init=1, max_iter=iters, tol=0.0,
                        algorithm="lloyd").fit(X, sample_weight=w)
        np.testing.assert_allclose(C, ref.cluster_centers_, rtol=1e-10, atol=1e-12)
        # sklearn's labels are the assignment to its final centres
        np.testing.assert_array_equal(KM.assign(X, C)[0], ref.labels_)


def test_one_dimensional_closed_form():
    X = np.array([[0.0], [1.0], [10.0], [11.0], [12.0]])
    C, W, a = KM.lloyd(X, None, np.array([[0.0], [10.0]]), 1)
    np.testing.assert_allclose(C[:, 0], [0.5, 11.0])
    np.testing.assert_array_equal(W, [2, 3])
    np.testing.assert_array_equal(a, [0, 0, 1, 1, 1])


def test_ties_go_to_the_lowest_index_and_empty_centres_stay():
    X = np.array([[1.0, 0.0], [2.0, 0.0], [0.0, 3.0]])
    C0 = np.array([[0.0, 0.0], [0.0, 0.0], [9.0, 9.0]])
    a, d2, margin = KM.assign(X, C0)
    np.testing.assert_array_equal(a, [0, 0, 0])
    np.testing.assert_array_equal(margin, [0.0, 0.0, 0.0])
    C, W, _ = KM.lloyd(X, None, C0, 1)
    np.testing.assert_allclose(C[0], X.mean(0))
    np.testing.assert_array_equal(C[1:], C0[1:])
    np.testing.assert_array_equal(W, [3, 0, 0])


def test_weights_equal_replicated_points():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((30, 5))
    reps = rng.integers(1, 4, 30)
    C0 = X[:4]
    Cw, Ww, _ = KM.lloyd(X, reps.astype(float), C0, 5)
    Cr, Wr, _ = KM.lloyd(np.repeat(X, reps, axis=0), None, C0, 5)
    np.testing.assert_allclose(Cw, Cr, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Ww, Wr)


def test_cost_never_increases():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((300, 6))
    w = rng.uniform(0.5, 2.0, 300)
    C = X[:12].copy()
    last = KM.cost(X, w, C)
    for _ in range(10):
        C, _, _ = KM.lloyd(X, w, C, 1)
        c = KM.cost(X, w, C)
        assert c <= last * (1 + 1e-12)
        last = c


def test_converged_partition_is_a_fixed_point():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((120, 3))
    C, W, a = KM.lloyd(X, None, X[:5], 60)
    a2, _, _ = KM.assign(X, C)
    np.testing.assert_array_equal(a, a2)
    for j in range(5):
        np.testing.assert_allclose(C[j], X[a == j].mean(0), rtol=1e-12)


def test_brute_force_optimum_on_separated_data():
    # three well separated pairs: the best 3-partition (by exhaustive search)
    # is what Lloyd reaches from one seed per pair
    X = np.array([[0, 0], [0, 1], [10, 0], [10, 1], [0, 20], [1, 20]], dtype=float)
    best = None
    for labels in itertools.product(range(3), repeat=6):
        labels = np.array(labels)
        if len(set(labels)) < 3:
            continue
        c = sum(((X[labels == j] - X[labels == j].mean(0)) ** 2).sum() for j in range(3))
        best = c if best is None or c < best else best
    C, _, _ = KM.lloyd(X, None, X[[0, 2, 4]], 5)
    assert abs(KM.cost(X, None, C) - best) < 1e-12


def test_micro_step_with_every_point_a_centre():
    rng = np.random.default_rng(5)
    F = rng.standard_normal((40, 8))
    out = KM.stream_kmeans(F, np.zeros((0, 8)), np.zeros(0), 40, np.arange(40), 3, 1)
    np.testing.assert_array_equal(out["micro"], F)
    np.testing.assert_array_equal(out["micro_w"], np.ones(40))
    np.testing.assert_array_equal(out["D"], F)


def test_stream_recovers_separated_clusters_and_conserves_weight():
    rng = np.random.default_rng(6)
    K, D = 6, 16
    protos = 10.0 * rng.standard_normal((K, D))
    # previous dictionary: near each prototype, weight 50 each
    D_prev = protos + 0.01 * rng.standard_normal((K, D))
    w_prev = np.full(K, 50.0)
    # new keyframe: 5 sub-blobs around each prototype, 20 points each
    sub = np.repeat(protos, 5, axis=0) + 0.3 * rng.standard_normal((5 * K, D))
    F = np.repeat(sub, 20, axis=0) + 0.01 * rng.standard_normal((5 * K * 20, D))
    seeds = np.arange(0, 5 * K * 20, 20)  # one seed per sub-blob
    out = KM.stream_kmeans(F, D_prev, w_prev, K, seeds, 4, 4)
    # micro-centres are the sub-blob means, with weight 20
    np.testing.assert_allclose(out["micro"], F.reshape(5 * K, 20, D).mean(1), rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(out["micro_w"], np.full(5 * K, 20.0))
    # each output centre is the weighted mean of its prototype's old centre and sub-blobs
    for j in range(K):
        pts = np.concatenate([D_prev[j:j + 1] * 50.0, F[j * 100:(j + 1) * 100]], axis=0)
        np.testing.assert_allclose(out["D"][j], pts.sum(0) / 150.0, rtol=1e-12, atol=1e-12)
    assert abs(out["W"].sum() - (w_prev.sum() + F.shape[0])) < 1e-9
    np.testing.assert_array_equal(out["W"], np.full(K, 150.0))


def test_stream_first_keyframe_starts_from_micro_centres():
    rng = np.random.default_rng(7)
    X, _ = _blobs(rng, 4, 25, 10)
    seeds = np.array([0, 25, 50, 75, 1, 26, 51, 76])
    out = KM.stream_kmeans(X, np.zeros((0, 10)), np.zeros(0), 4, seeds, 3, 3)
    # global init = the first 4 micro-centres, one per blob -> blob means
    np.testing.assert_allclose(out["D"], X.reshape(4, 25, 10).mean(1), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["W"], np.full(4, 25.0))


def test_stream_argument_checks():
    F = np.zeros((10, 4))
    with pytest.raises(ValueError):
        KM.stream_kmeans(F, np.zeros((5, 4)), np.ones(5), 4, np.arange(3), 1, 1)
    with pytest.raises(ValueError):
        KM.stream_kmeans(F, np.zeros((0, 4)), np.zeros(0), 4, np.arange(3), 1, 1)
    with pytest.raises(ValueError):
        KM.lloyd(F, None, F[:2], 0)
