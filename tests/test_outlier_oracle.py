"""Pins of the oracle's proximity-based outlier scores (Section 4, large-scale outlier detection):
closed forms on a lattice, exact duplicates, planted outliers, and an independent float64
brute-force computation."""
import numpy as np

import oracle


def test_lattice_closed_forms():
    n = 50
    P = np.arange(n, dtype=np.float32).reshape(n, 1)
    s2, o2 = oracle.outlier_scores(P, 2)
    want2 = np.ones(n, dtype=np.float32)
    want2[[0, n - 1]] = 1.5  # an end point's two nearest others are 1 and 2 away
    assert np.array_equal(s2, want2)
    assert list(o2[:2]) == [0, n - 1] and list(o2[2:]) == list(range(1, n - 1))
    s3, _ = oracle.outlier_scores(P, 3)
    want3 = np.full(n, np.float32(4.0 / 3.0))
    want3[[0, n - 1]] = np.float32(2.0)  # 1, 2, 3
    assert np.array_equal(s3, want3)


def test_duplicates_and_a_missing_own_entry():
    P = np.array([[0.0], [0.0], [10.0], [11.0]], dtype=np.float32)
    s, o = oracle.outlier_scores(P, 1)
    assert np.array_equal(s, np.array([0, 0, 1, 1], dtype=np.float32))
    assert list(o) == [2, 3, 0, 1]
    # four copies of one point, k = 1: point 3's two nearest are copies 0 and 1 (smaller
    # indices win ties), so its own entry is absent and the first one is kept
    Q = np.zeros((4, 2), dtype=np.float32)
    s, o = oracle.outlier_scores(Q, 1)
    assert np.array_equal(s, np.zeros(4, dtype=np.float32)) and list(o) == [0, 1, 2, 3]


def test_planted_outliers_rank_first():
    rng = np.random.default_rng(11)
    base = rng.standard_normal((2000, 5)).astype(np.float32)
    far = np.zeros((5, 5), dtype=np.float32)
    radii = [50.0, 90.0, 70.0, 60.0, 80.0]
    for i, r in enumerate(radii):
        far[i, i] = r
    P = np.vstack([base, far])
    s, o = oracle.outlier_scores(P, 10)
    planted = 2000 + np.argsort(radii)[::-1]
    assert list(o[:5]) == list(planted)
    for i, r in enumerate(radii):
        assert abs(float(s[2000 + i]) - r) < 5.0


def test_matches_float64_brute_force():
    rng = np.random.default_rng(12)
    P = rng.standard_normal((300, 3)).astype(np.float32)
    k = 4
    s, _ = oracle.outlier_scores(P, k)
    idx, d2 = oracle.brute_f64(P, P, k + 1)
    want = np.empty(len(P))
    for i in range(len(P)):
        keep = [j for j in range(k + 1) if idx[i, j] != i][:k]
        want[i] = np.mean(np.sqrt(d2[i, keep]))
    np.testing.assert_allclose(s, want, rtol=1e-5)
