"""Evaluation helpers (not the method): R_NX curve and its AUC."""
import numpy as np

from inputs.knn_metrics import rnx_auc, rnx_curve, rnx_points


def test_rnx_perfect_and_random():
    rng = np.random.default_rng(0)
    N, n, K = 5000, 200, 32
    exact = np.stack([rng.choice(N, K, replace=False) for _ in range(n)])
    r = rnx_curve(exact, exact, N)
    np.testing.assert_allclose(r, 1.0)
    assert abs(rnx_auc(r) - 1.0) < 1e-12
    rand = np.stack([rng.choice(N, K, replace=False) for _ in range(n)])
    r0 = rnx_curve(rand, exact, N)
    assert abs(rnx_auc(r0)) < 0.02


def test_rnx_matches_set_definition():
    """Q_NX(K) counted directly from the K-prefix sets."""
    rng = np.random.default_rng(1)
    N, n, K = 300, 40, 16
    exact = np.stack([rng.permutation(N)[:K] for _ in range(n)])
    est = exact.copy()
    for r in range(n):       # shuffle some entries and replace a few
        est[r] = rng.permutation(est[r])
        est[r, rng.integers(0, K, 3)] = rng.integers(0, N, 3)
    got = rnx_curve(est, exact, N)
    for k in range(1, K + 1):
        q = np.mean([len(set(est[r, :k]) & set(exact[r, :k])) / k for r in range(n)])
        want = ((N - 1) * q - k) / (N - 1 - k)
        assert abs(got[k - 1] - want) < 1e-12


def test_rnx_points_rows_and_mean():
    """Each row from its own K-prefix sets; the rows average to rnx_curve."""
    rng = np.random.default_rng(2)
    N, n, K = 400, 30, 12
    exact = np.stack([rng.permutation(N)[:K] for _ in range(n)])
    est = np.stack([rng.permutation(np.concatenate([e[:8], rng.choice(
        np.setdiff1d(np.arange(N), e), 4, replace=False)])) for e in exact])
    pts = rnx_points(est, exact, N)
    for r in range(n):
        for k in range(1, K + 1):
            q = len(set(est[r, :k]) & set(exact[r, :k])) / k
            assert abs(pts[r, k - 1] - ((N - 1) * q - k) / (N - 1 - k)) < 1e-12
    np.testing.assert_allclose(pts.mean(axis=0), rnx_curve(est, exact, N), atol=1e-12)
