"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-type the oracle's own formulas: each checks the oracle
against an independent fact (published known answers, finite differences of
the cost, closed-form limits, brute force, statistical identities).
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from inputs.generators import blobs, y_init

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- counter-based generator ------------------------------------------------
def test_philox_known_answers(oracle_lib):
    """Philox4x32-10 reproduces the published known-answer vectors."""
    O = oracle_lib
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


# --- exact cost and gradient (eqs. (4), (5)) --------------------------------
def _small_problem(N=40, D=6, d=2, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(N, D)).astype(np.float32)
    Y = rng.normal(scale=2.0, size=(N, d))
    return X, Y


@pytest.mark.parametrize("alpha", [0.3, 0.5, 1.0, 2.0, 4.0])
def test_exact_gradient_matches_finite_differences(oracle_lib, alpha):
    """Eq. (5) is the derivative of KL(P||Q) with Q from eq. (4)."""
    O = oracle_lib
    X, Y = _small_problem(N=30, d=3)
    P, _ = O.exact_P(X, 5.0)
    G = O.exact_grad(P, Y, alpha)
    h = 1e-6
    rng = np.random.default_rng(11)
    for _ in range(12):
        i, c = rng.integers(30), rng.integers(3)
        Yp, Ym = Y.copy(), Y.copy()
        Yp[i, c] += h
        Ym[i, c] -= h
        fd = (O.exact_cost(P, Yp, alpha) - O.exact_cost(P, Ym, alpha)) / (2 * h)
        assert abs(fd - G[i, c]) <= 1e-6 * max(1.0, np.abs(G).max()), (i, c, fd, G[i, c])


def test_alpha_one_is_tsne(oracle_lib):
    """At alpha = 1, eq. (5) equals the t-SNE gradient of eq. (3) with Cauchy q of eq. (2)."""
    O = oracle_lib
    X, Y = _small_problem()
    P, _ = O.exact_P(X, 8.0)
    G = O.exact_grad(P, Y, 1.0)
    diff = Y[:, None, :] - Y[None, :, :]
    k = 1.0 / (1.0 + (diff ** 2).sum(-1))
    np.fill_diagonal(k, 0.0)
    Q = k / k.sum()
    G3 = 4.0 * (((P - Q) * k)[:, :, None] * diff).sum(1)
    np.testing.assert_allclose(G, G3, rtol=1e-10, atol=1e-14)


def test_large_alpha_is_gaussian_sne(oracle_lib):
    """As alpha grows, w -> exp(-d^2) and w^(1/alpha) -> 1 (symmetric SNE gradient)."""
    O = oracle_lib
    X, Y = _small_problem()
    Y = Y * 0.3
    P, _ = O.exact_P(X, 8.0)
    G = O.exact_grad(P, Y, 1e6)
    diff = Y[:, None, :] - Y[None, :, :]
    g = np.exp(-(diff ** 2).sum(-1))
    np.fill_diagonal(g, 0.0)
    Q = g / g.sum()
    Gs = 4.0 * ((P - Q)[:, :, None] * diff).sum(1)
    assert np.linalg.norm(G - Gs) <= 1e-4 * np.linalg.norm(Gs)


# --- perplexity calibration (eq. (1)) ----------------------------------------
def test_calibration_hits_the_perplexity(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(5)
    for K, perp in [(32, 10.0), (64, 20.0), (16, 3.0), (32, 31.0), (8, 1.5)]:
        for scale in [1e-3, 1.0, 50.0, 1e4]:
            d2 = np.sort(rng.gamma(3.0, scale, size=K))
            (beta, m, r, invS), noroot = O.calibrate(d2, perp)
            assert not noroot
            p = np.exp(-beta * (d2 - d2.min()))
            p /= p.sum()
            H = -(p[p > 0] * np.log(p[p > 0])).sum()
            assert abs(H - np.log(perp)) < 1e-9, (K, perp, scale, H)
            assert m == d2.min() and r == d2.max()
            assert abs(invS * np.exp(-beta * (d2 - m)).sum() - 1.0) < 1e-12


def test_calibration_degenerate_rows(oracle_lib):
    O = oracle_lib
    # all distances equal: any beta gives the uniform row, entropy ln K > ln perp
    (beta, m, r, invS), noroot = O.calibrate(np.full(16, 2.0), 5.0)
    assert beta == 0.0 and noroot and abs(invS - 1 / 16) < 1e-15
    # 8 ties at the minimum with ln 8 > ln 5: no finite root, row uniform over the ties
    d2 = np.concatenate([np.zeros(8), np.linspace(1, 2, 8)])
    (beta, m, r, invS), noroot = O.calibrate(d2, 5.0)
    assert noroot and beta == 1e30 and abs(invS - 1 / 8) < 1e-15
    # exactly perplexity-many ties: the entropy only reaches ln perp in the limit
    d2 = np.concatenate([np.zeros(5), np.linspace(1, 2, 11)])
    (beta, m, r, invS), noroot = O.calibrate(d2, 5.0)
    assert noroot and beta == 1e30 and abs(invS - 1 / 5) < 1e-15
    # one tie fewer: a finite root exists and hits the target entropy
    d2 = np.concatenate([np.zeros(4), np.linspace(1e-3, 2, 12)])
    (beta, m, r, invS), noroot = O.calibrate(d2, 5.0)
    p = invS * np.exp(-beta * (d2 - m))
    assert not noroot and beta < 1e30
    assert abs(-(p[p > 0] * np.log(p[p > 0])).sum() - np.log(5.0)) < 1e-9


# --- the method step with complete lists equals the exact gradient ----------
def _complete_state(O, N=24, D=5, d=2, alpha=1.0, perp=6.0, seed=9):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(N, D)).astype(np.float32)
    Y0 = rng.normal(scale=1.5, size=(N, d)).astype(np.float32)
    S = O.OracleState(X, d, N - 1, N - 1, 77, Y0)
    hp = O.Hyper(alpha=alpha, perplexity=perp, lr=3.0, momentum=0.0, attr=1.0, rep=1.0, n_neg=5,
                 hd_mode=1)
    S.init(hp)
    return X, S, hp


@pytest.mark.parametrize("alpha", [0.5, 1.0, 3.0])
@pytest.mark.parametrize("N", [24, 200])
def test_complete_lists_give_exact_affinities_and_gradient(oracle_lib, alpha, N):
    """With K_hd = N-1 the three sets of eq. (6) are exhaustive and nothing is
    sampled (N = 200: lists of 199, longer than a wave)."""
    O = oracle_lib
    X, S, hp = _complete_state(O, N=N, alpha=alpha, perp=6.0 if N < 100 else 40.0)
    hp = hp.copy(alpha=alpha)
    Pex, beta_ex = O.exact_P(X, hp.perplexity)
    # sparse affinities in dense form
    Pd = np.zeros((N, N))
    for i in range(N):
        Pd[i, S.hd_idx[i]] = S.P[i]
    np.testing.assert_allclose(Pd, Pex, rtol=1e-12, atol=1e-16)
    assert abs(Pd.sum() - 1.0) < 1e-12
    np.testing.assert_allclose(S.beta[:N], beta_ex, rtol=1e-12)
    Y0 = S.Y[:N].copy()
    st = S.step(hp, want_partials=True)
    assert st["fired"] == 1 and st["n_new"] == 0   # nothing can enter a complete list
    g = 4.0 * (hp.attr * st["A"] - hp.rep * st["R"] / st["Z"])
    Gex = O.exact_grad(Pex, Y0, alpha)
    np.testing.assert_allclose(g, Gex, rtol=1e-9, atol=1e-12 * np.abs(Gex).max())
    # Z is the full sum over ordered pairs of eq. (4)
    diff = Y0[:, None, :] - Y0[None, :, :]
    w = (1.0 + (diff ** 2).sum(-1) / alpha) ** (-alpha)
    np.fill_diagonal(w, 0.0)
    assert abs(st["Z"] - w.sum()) <= 1e-12 * w.sum()
    # momentum 0: plain gradient descent
    np.testing.assert_allclose(S.Y[:N], Y0 - hp.lr * Gex, rtol=1e-9, atol=1e-12)


def test_momentum_update(oracle_lib):
    """V <- mu V - lr g; Y <- Y + V."""
    O = oracle_lib
    N = 24
    X, S, hp = _complete_state(O, N=N)
    hp = hp.copy(momentum=0.7)
    S.V[:N] = np.random.default_rng(1).normal(size=(N, 2))
    V0, Y0 = S.V[:N].copy(), S.Y[:N].copy()
    Pex, _ = O.exact_P(X, hp.perplexity)
    st = S.step(hp)
    Gex = O.exact_grad(Pex, Y0, hp.alpha)
    V1 = 0.7 * V0 - hp.lr * Gex
    np.testing.assert_allclose(S.V[:N], V1, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(S.Y[:N], Y0 + V1, rtol=1e-9, atol=1e-12)


def test_attraction_repulsion_scales(oracle_lib):
    """g = 4 (a A - r R / Z): the two parts are kept apart and scaled separately."""
    O = oracle_lib
    N = 24
    X, S, hp = _complete_state(O, N=N)
    Pex, _ = O.exact_P(X, hp.perplexity)
    Y0 = S.Y[:N].copy()
    S2 = S.copy()
    st = S.step(hp.copy(attr=3.0, rep=0.5), want_partials=True)
    diff = Y0[:, None, :] - Y0[None, :, :]
    k = 1.0 / (1.0 + (diff ** 2).sum(-1))
    np.fill_diagonal(k, 0.0)
    Z = k.sum()
    att = 4 * ((Pex * k)[:, :, None] * diff).sum(1)
    rep = 4 * ((k * k / Z)[:, :, None] * diff).sum(1)
    np.testing.assert_allclose(S.Y[:N], Y0 - hp.lr * (3.0 * att - 0.5 * rep), rtol=1e-9,
                               atol=1e-12)
    del S2


# --- negative sampling (Sec. 2.3 and eq. (6)) --------------------------------
def test_negative_sampling_is_unbiased(oracle_lib):
    """Averaged over draws, the sampled rest term equals the exact sum over j outside U."""
    O = oracle_lib
    N, d, K = 300, 2, 8
    rng = np.random.default_rng(2)
    X = rng.normal(size=(N, 4)).astype(np.float32)
    Y = rng.normal(scale=3.0, size=(N, d)).astype(np.float32)
    S = O.OracleState(X, d, K, K, 5, Y)
    hp = O.Hyper(alpha=0.7, perplexity=4.0, n_neg=6, hd_mode=2)
    S.init(hp)
    # exact lists in both spaces so the LD refinement cannot change U
    ex, exd = O.knn_exact(X, np.arange(N), K)
    S.hd_idx[:N], S.hd_d2[:N] = ex, exd
    Yd = np.ascontiguousarray(Y.astype(np.float64))
    dd = ((Yd[:, None, :] - Yd[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(dd, np.inf)
    S.ld_idx[:N] = np.argsort(dd, axis=1, kind="stable")[:, :K]
    for i in range(N):
        S.P[i] = S.psym_row(i)
    i = 17
    U = set(S.hd_idx[i]) | set(S.ld_idx[i])
    alpha = hp.alpha
    yi = S.Y[i]
    exact_R = np.zeros(d)
    exact_Z = 0.0
    U_R = np.zeros(d)
    U_Z = 0.0
    for j in range(N):
        if j == i:
            continue
        q2 = ((yi - S.Y[j]) ** 2).sum()
        w = (1 + q2 / alpha) ** (-alpha)
        wa = 1 / (1 + q2 / alpha)
        if j in U:
            U_R += w * wa * (yi - S.Y[j])
            U_Z += w
        else:
            exact_R += w * wa * (yi - S.Y[j])
            exact_Z += w
    T = 4000
    est_Z = np.zeros(T)
    est_R = np.zeros((T, d))
    for t in range(T):
        ld, A, R, Zh = S.ld_refine_grad_point(hp, i, t)
        assert set(ld) == set(S.ld_idx[i])
        est_Z[t] = Zh - U_Z
        est_R[t] = R - U_R
    z = (est_Z.mean() - exact_Z) / (est_Z.std() / np.sqrt(T))
    assert abs(z) < 4.5, z
    for c in range(d):
        zc = (est_R[:, c].mean() - exact_R[c]) / (est_R[:, c].std() / np.sqrt(T))
        assert abs(zc) < 4.5, zc


# --- KNN refinement (Sec. 3, Sec. 4.1) ---------------------------------------
def test_knn_exact_matches_brute_force_numpy(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(4)
    X = rng.normal(size=(500, 7)).astype(np.float32)
    q = np.array([0, 5, 99, 499])
    idx, d2 = O.knn_exact(X, q, 10)
    Xd = X.astype(np.float64)
    for a, i in enumerate(q):
        dd = ((Xd - Xd[i]) ** 2).sum(1)
        dd[i] = np.inf
        order = np.lexsort((np.arange(500), dd))[:10]
        assert list(idx[a]) == list(order)
        np.testing.assert_allclose(d2[a], dd[order], rtol=1e-15)


def test_refinement_lists_are_valid_and_improve(oracle_lib):
    """Lists stay sorted, unique and self-free; each HD list's K-th distance never grows."""
    O = oracle_lib
    X, lab = blobs(n_clusters=5, per_cluster=80, D=10, seed=21)
    N, K = X.shape[0], 16
    S = O.OracleState(X, 2, K, 8, 123, y_init(N, 2))
    hp = O.Hyper(alpha=1.0, perplexity=5.0, lr=N / 12, momentum=0.5, attr=12.0, n_neg=4,
                 hd_mode=1)
    S.init(hp)
    Xd = X.astype(np.float64)
    prev_kth = S.hd_d2[:N, -1].copy()
    for it in range(60):
        st = S.step(hp)
        hd, d2, ld = S.hd_idx[:N], S.hd_d2[:N], S.ld_idx[:N]
        assert np.all(np.diff(d2, axis=1) >= 0)
        for i in range(0, N, 7):
            assert len(set(hd[i])) == K and i not in set(hd[i])
            assert len(set(ld[i])) == 8 and i not in set(ld[i])
            np.testing.assert_allclose(d2[i], ((Xd[hd[i]] - Xd[i]) ** 2).sum(1), rtol=1e-12)
        kth = d2[:, -1]
        assert np.all(kth <= prev_kth)
        assert st["n_new"] == int(np.sum(S.flags[:N]))
        prev_kth = kth.copy()
    ex, _ = O.knn_exact(X, np.arange(N), K)
    recall = np.mean([len(set(S.hd_idx[i]) & set(ex[i])) for i in range(N)]) / K
    assert recall > 0.97, recall


def test_refined_lists_converge_to_exact(oracle_lib):
    """On a tiny set the interleaved refinement finds the exact K-NN sets."""
    O = oracle_lib
    X, _ = blobs(n_clusters=3, per_cluster=40, D=5, seed=8)
    N, K = X.shape[0], 8
    S = O.OracleState(X, 2, K, 6, 9, y_init(N, 2))
    hp = O.Hyper(alpha=1.0, perplexity=4.0, lr=N / 12, momentum=0.5, attr=4.0, n_neg=4,
                 hd_mode=1)
    S.init(hp)
    for _ in range(300):
        S.step(hp)
    ex, exd = O.knn_exact(X, np.arange(N), K)
    np.testing.assert_array_equal(S.hd_idx[:N], ex)
    np.testing.assert_allclose(S.hd_d2[:N], exd, rtol=1e-15)


def test_ld_lists_converge_to_exact_in_a_fixed_embedding(oracle_lib):
    """With the learning rate at 0 the embedding stays where it is, and the
    LD refinement (old list plus candidates, kept by distance in Y) must end
    on the exact K_ld nearest neighbours in Y, nearest first."""
    O = oracle_lib
    X, _ = blobs(n_clusters=3, per_cluster=50, D=6, seed=12)
    N, Kh, Kl = X.shape[0], 10, 7
    Y0 = np.random.default_rng(4).normal(size=(N, 3))
    S = O.OracleState(X, 3, Kh, Kl, 17, Y0).init(
        O.Hyper(alpha=1.0, perplexity=5.0, lr=0.0, momentum=0.5, n_neg=4, hd_mode=0))
    hp = O.Hyper(alpha=1.0, perplexity=5.0, lr=0.0, momentum=0.5, n_neg=4, hd_mode=0)
    for _ in range(250):
        S.step(hp)
    Y = S.live("Y")
    np.testing.assert_array_equal(Y, Y0)
    d2 = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    exact = np.argsort(d2, axis=1, kind="stable")[:, :Kl]
    np.testing.assert_array_equal(S.live("ld_idx"), exact)


# --- refinement probability and its smoothing (Sec. 3) -----------------------
def test_coin_probability(oracle_lib):
    O = oracle_lib
    assert all(O.coin(1.0, t, 42) for t in range(200))          # E = 1 -> p = 1
    fr = np.mean([O.coin(0.0, t, 42) for t in range(40000)])   # E = 0 -> p = 0.05
    assert abs(fr - 0.05) < 4 * np.sqrt(0.05 * 0.95 / 40000)
    fr = np.mean([O.coin(0.5, t, 7) for t in range(40000)])    # p = 0.525
    assert abs(fr - 0.525) < 4 * np.sqrt(0.525 * 0.475 / 40000)
    assert O.coin(0.0, 3, 42, hd_mode=1) == 1 and O.coin(1.0, 3, 42, hd_mode=2) == 0


def test_coin_margin_decides_the_coin(oracle_lib):
    """The coin fires exactly when the draw lies below p 2^32, p = 0.05 + 0.95 E."""
    O = oracle_lib
    for E in (0.0, 0.013, 0.5, 0.97):
        for t in range(300):
            m = O.coin_margin(E, t, 42)
            assert O.coin(E, t, 42) == (m < 0)
            # the margin is the draw minus the threshold: recover the draw
            u = m + (0.05 + 0.95 * E) * 2.0 ** 32
            assert abs(u - round(u)) < 1e-6 and 0 <= round(u) < 2 ** 32


def test_E_smoothing(oracle_lib):
    O = oracle_lib
    assert O.E_next(1.0, 0, 100, 0.1) == 0.9
    assert O.E_next(0.5, 100, 100, 0.25) == 0.625
    e = 1.0
    for _ in range(400):
        e = O.E_next(e, 30, 100, 0.1)
    assert abs(e - 0.3) < 1e-15                                  # fixed point N_new / N


# --- determinism ----------------------------------------------------------------
_DET = r"""
import numpy as np, sys
sys.path.insert(0, %r)
from oracle import oracle as O
from inputs.generators import blobs, y_init
X, _ = blobs(n_clusters=4, per_cluster=60, D=8, seed=3)
S = O.OracleState(X, 2, 12, 8, 5, y_init(240, 2))
hp = O.Hyper(perplexity=5.0, lr=20.0, attr=4.0, n_neg=4)
S.init(hp)
for _ in range(20): S.step(hp)
sys.stdout.write(S.Y[:240].tobytes().hex()[:4000] + S.hd_idx[:240].tobytes().hex()[:4000])
"""


def test_thread_count_independence():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for nt in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        outs.append(subprocess.check_output([sys.executable, "-c", _DET % root], env=env))
    assert outs[0] == outs[1]


# --- dynamic data ------------------------------------------------------------------
def test_insert_and_drift(oracle_lib):
    O = oracle_lib
    X, _ = blobs(n_clusters=4, per_cluster=60, D=8, seed=3)
    N0 = 200
    S = O.OracleState(X[:N0], 2, 12, 8, 5, y_init(N0, 2), capacity=240)
    hp = O.Hyper(perplexity=5.0, lr=20.0, attr=4.0, n_neg=4, hd_mode=1)
    S.init(hp)
    for _ in range(10):
        S.step(hp)
    S.insert(hp, X[N0:], np.zeros((40, 2)))
    assert S.N == 240
    Xd = X.astype(np.float64)
    for i in range(N0, 240):
        assert len(set(S.hd_idx[i])) == 12 and i not in set(S.hd_idx[i])
        np.testing.assert_allclose(S.hd_d2[i], ((Xd[S.hd_idx[i]] - Xd[i]) ** 2).sum(1), rtol=1e-12)
        assert S.flags[i] == 1
    assert abs(S.P[:240].sum() - S.copy().P[:240].sum()) == 0
    # drift: move 5 points; every list entry involving them gets its new distance
    ids = np.array([3, 50, 120, 201, 239])
    Xn = X[ids] + 0.5
    S.drift(hp, ids, Xn)
    Xd = S.X[:240].astype(np.float64)
    for i in range(240):
        np.testing.assert_allclose(S.hd_d2[i], ((Xd[S.hd_idx[i]] - Xd[i]) ** 2).sum(1),
                                   rtol=1e-12)
        assert np.all(np.diff(S.hd_d2[i]) >= 0)
    assert np.all(S.V[ids] == 0)
    for _ in range(5):
        S.step(hp)


# --- jump start by a random linear projection --------------------------------
def _js_state(O, X, d=3, seed=5):
    N = X.shape[0]
    S = O.OracleState(X, d, 8, 8, seed, np.zeros((N, d), np.float32))
    return S


def test_jump_start_centring_scale_and_distances(oracle_lib):
    """Centred (mean exactly 0), each coordinate of variance about sigma^2 on
    isotropic data, and squared distances preserved on average up to the
    factor d s^2 of a +-1 projection (Johnson-Lindenstrauss)."""
    O = oracle_lib
    rng = np.random.default_rng(3)
    N, D, d, sigma = 6000, 48, 3, 0.05
    X = (rng.normal(size=(N, D)) * 2.0 + 7.0).astype(np.float32)
    S = _js_state(O, X, d)
    S.jump_start(0, sigma)
    Y = S.live("Y")
    assert np.all(S.live("V") == 0.0)
    assert np.all(np.abs(Y.mean(0)) < 1e-12 * sigma * N)
    assert np.all(np.abs(Y.std(0) / sigma - 1.0) < 0.06), Y.std(0) / sigma
    Xc = X.astype(np.float64) - X.astype(np.float64).mean(0)
    s2 = sigma ** 2 / (Xc ** 2).sum(1).mean()
    a, b = rng.integers(0, N, 4000), rng.integers(0, N, 4000)
    keep = a != b
    ratio = ((Y[a] - Y[b]) ** 2).sum(1)[keep] / (d * s2 * ((Xc[a] - Xc[b]) ** 2).sum(1)[keep])
    assert abs(ratio.mean() - 1.0) < 0.05, ratio.mean()


def test_jump_start_invariances_and_projections(oracle_lib):
    """Shifting or rescaling the data leaves the projection unchanged; the
    projection index selects a different sign matrix; a constant data set
    maps to 0."""
    O = oracle_lib
    rng = np.random.default_rng(4)
    X = rng.normal(size=(500, 20)).astype(np.float32)
    S = _js_state(O, X)
    S.jump_start(0, 1.0)
    Y0 = S.live("Y").copy()
    S2 = _js_state(O, X * np.float32(4.0))
    S2.jump_start(0, 1.0)
    np.testing.assert_allclose(S2.live("Y"), Y0, rtol=1e-12, atol=1e-12)
    S3 = _js_state(O, X + np.float32(0.5))
    S3.jump_start(0, 1.0)
    np.testing.assert_allclose(S3.live("Y"), Y0, rtol=1e-5, atol=1e-5)
    S.jump_start(1, 1.0)
    assert not np.allclose(S.live("Y"), Y0)
    S.jump_start(0, 1.0)
    np.testing.assert_array_equal(S.live("Y"), Y0)
    S4 = _js_state(O, np.ones((50, 20), np.float32))
    S4.jump_start(0, 1.0)
    assert np.all(S4.live("Y") == 0.0)


# --- point deletion ------------------------------------------------------------
def test_delete_keeps_a_consistent_state(oracle_lib):
    """After deleting points every list entry is a live point other than the
    row's own, rows are unique and sorted by (d2, id), every HD distance is
    the true distance between the renumbered rows, survivors keep their
    coordinates, and recalibrated rows hit the perplexity."""
    O = oracle_lib
    rng = np.random.default_rng(8)
    N, D, d, Kh, Kl, perp = 600, 12, 2, 16, 8, 5.0
    X = rng.normal(size=(N, D)).astype(np.float32)
    Y0 = rng.normal(size=(N, d)).astype(np.float32)
    hp = O.Hyper(perplexity=perp, lr=50.0, n_neg=4, hd_mode=1)
    S = O.OracleState(X, d, Kh, Kl, 9, Y0).init(hp)
    for _ in range(5):
        S.step(hp)
    Yb, Xb = S.live("Y").copy(), S.live("X").copy()
    ids = rng.choice(N, 90, replace=False)
    newid = S.delete(hp, ids)
    N1 = N - 90
    assert S.N == N1
    alive = newid >= 0
    assert alive.sum() == N1 and np.all(newid[ids] == -1)
    np.testing.assert_array_equal(np.sort(newid[alive]), np.arange(N1))
    np.testing.assert_array_equal(S.live("Y")[newid[alive]], Yb[alive])
    np.testing.assert_array_equal(S.live("X")[newid[alive]], Xb[alive])
    H, Hd, L = S.live("hd_idx"), S.live("hd_d2"), S.live("ld_idx")
    for i in range(N1):
        for row in (H[i], L[i]):
            assert np.all((row >= 0) & (row < N1)) and i not in row
            assert len(set(row.tolist())) == row.size
        Xl = S.live("X").astype(np.float64)
        true = ((Xl[H[i]] - Xl[i]) ** 2).sum(1)
        np.testing.assert_allclose(Hd[i], true, rtol=1e-12, atol=1e-12)
        order = np.lexsort((H[i], Hd[i]))
        np.testing.assert_array_equal(order, np.arange(Kh))
    flagged = np.nonzero(S.live("flags") == 1)[0]
    assert flagged.size > 0
    for i in flagged[:50]:
        p = np.exp(-S.beta[i] * (Hd[i] - S.m[i])) * S.invS[i]
        assert abs(-(p * np.log(p)).sum() - np.log(perp)) < 1e-8
    assert S.live("P").sum() <= 1.0 + 1e-9
    S.step(hp)          # the state still steps
    assert np.all(np.isfinite(S.live("Y")))


# --- clustering for the hierarchy graph ----------------------------------------
def test_cluster_equals_dbscan_on_exact_lists(oracle_lib):
    """With exact LD neighbour lists holding every eps-neighbour, the clusters
    are DBSCAN's (scikit-learn): same noise, same partition of the core
    points, border points in the cluster of a core point within eps."""
    from sklearn.cluster import DBSCAN

    O = oracle_lib
    rng = np.random.default_rng(12)
    d, K, min_pts = 4, 48, 5
    cent = rng.normal(scale=12.0, size=(5, d))
    Y = np.concatenate([c + rng.normal(scale=s, size=(250, d))
                        for c, s in zip(cent, (0.3, 0.4, 0.5, 0.4, 0.3))] +
                       [rng.uniform(-25, 25, size=(60, d))])
    Y = Y.astype(np.float32).astype(np.float64)
    N = Y.shape[0]
    D2 = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(D2, np.inf)
    knn = np.argsort(D2, axis=1, kind="stable")[:, :K]
    eps = 0.33
    assert ((D2 <= eps * eps).sum(1) <= K).all()           # lists hold every eps-neighbour
    assert np.abs(np.sqrt(D2[np.isfinite(D2)]) - eps).min() > 1e-5   # no pair at the boundary
    S = O.OracleState(np.zeros((N, 3), np.float32), d, 8, K, 1, Y.astype(np.float32))
    S.ld_idx[:N] = knn
    labels, nc = S.cluster(eps, min_pts)
    ref = DBSCAN(eps=eps, min_samples=min_pts).fit(Y)
    core = np.zeros(N, bool)
    core[ref.core_sample_indices_] = True
    np.testing.assert_array_equal(labels == -1, ref.labels_ == -1)
    assert nc == len(set(ref.labels_[core]))
    pairs = {(a, b) for a, b in zip(labels[core], ref.labels_[core])}
    assert len(pairs) == nc                                   # a one-to-one renaming
    for i in np.nonzero(~core & (labels >= 0))[0]:
        near = core & (D2[i] <= eps * eps)
        assert labels[i] in set(labels[near])
    assert nc > 5 and core.sum() > 500
    # clusters are numbered by the smallest index among their core points
    firsts = [np.nonzero((labels == k) & core)[0].min() for k in range(nc)]
    assert firsts == sorted(firsts)


# --- HD metric (Sec. 3: HD-side settings such as the metric may change) ----
def _rescaled_blobs(n_clusters, per_cluster, D, seed):
    """Blobs with every row scaled by a power of two (exact in FP32): the
    angular neighbours are the blobs', the Euclidean ones are not."""
    X, lab = blobs(n_clusters=n_clusters, per_cluster=per_cluster, D=D, seed=seed)
    rng = np.random.default_rng(seed + 1)
    X = (X * np.exp2(rng.integers(-3, 4, size=(X.shape[0], 1)))).astype(np.float32)
    return X, lab


def test_angular_metric_closed_forms_and_scipy(oracle_lib):
    """Angular delta^2 = |x/|x| - y/|y||^2 = 2 (1 - cos): right angles,
    parallel and opposite rows, 60 degrees, the zero row, SciPy's cosine
    distance (FP32 and BF16 rows), invariance to positive row scales."""
    from scipy.spatial.distance import cosine

    from inputs.generators import bf16_bits_to_f32, f32_to_bf16_bits
    O = oracle_lib
    e = np.eye(4, dtype=np.float32)
    X = np.stack([e[0], e[1], 3 * e[0], -2 * e[0], np.zeros(4, np.float32),
                  np.array([0.5, np.sqrt(0.75), 0, 0], np.float32)])

    def dm(a, b, Z=X):
        return O.hd_dist2(Z, a, b, metric=1)
    assert abs(dm(0, 1) - 2.0) < 1e-15
    assert abs(dm(0, 2)) < 1e-15
    assert abs(dm(0, 3) - 4.0) < 1e-15
    assert abs(dm(0, 4) - 1.0) < 1e-15 and dm(4, 4) == 0.0
    assert abs(dm(0, 5) - 1.0) < 1e-7
    assert O.hd_dist2(X, 0, 2) == 4.0           # metric 0 is still Euclidean
    rng = np.random.default_rng(5)
    R = rng.normal(size=(30, 17)).astype(np.float32)
    B = f32_to_bf16_bits(R)
    Rb = bf16_bits_to_f32(B).astype(np.float64)
    for a, b in [(0, 1), (2, 9), (17, 4), (29, 28)]:
        want = 2.0 * cosine(R[a].astype(np.float64), R[b].astype(np.float64))
        assert abs(dm(a, b, R) - want) < 1e-12
        assert abs(dm(a, b, B) - 2.0 * cosine(Rb[a], Rb[b])) < 1e-12
    Rs = (R * np.exp2(rng.integers(-6, 7, size=(30, 1)))).astype(np.float32)
    for a, b in [(0, 1), (5, 6), (11, 20)]:
        assert abs(dm(a, b, Rs) - dm(a, b, R)) < 1e-14


def test_angular_refinement_converges_to_exact_angular_knn(oracle_lib):
    """With metric 1 from the start, the interleaved refinement finds the
    exact K-NN sets of the angular distance (brute force with SciPy)."""
    from scipy.spatial.distance import cdist
    O = oracle_lib
    X, _ = _rescaled_blobs(3, 40, 5, 8)
    N, K = X.shape[0], 8
    S = O.OracleState(X, 2, K, 6, 9, y_init(N, 2), metric=1)
    hp = O.Hyper(alpha=1.0, perplexity=4.0, lr=N / 12, momentum=0.5, attr=4.0, n_neg=4,
                 hd_mode=1)
    S.init(hp)
    for _ in range(300):
        S.step(hp)
    A = 2.0 * cdist(X.astype(np.float64), X.astype(np.float64), "cosine")
    np.fill_diagonal(A, np.inf)
    ex = np.argsort(A, axis=1, kind="stable")[:, :K]
    np.testing.assert_array_equal(S.hd_idx[:N], ex)
    np.testing.assert_allclose(S.hd_d2[:N], np.take_along_axis(A, ex, 1), rtol=1e-12, atol=1e-15)
    # the Euclidean lists of the same rows differ
    exe, _ = O.knn_exact(X, np.arange(N), K)
    assert np.mean([len(set(a) & set(b)) for a, b in zip(ex, exe)]) < 0.8 * K


def test_metric_switch_recomputes_every_list(oracle_lib):
    """A switch keeps each list's members, gives every entry its distance in
    the new metric, re-sorts by (d2, id), flags and recalibrates every row
    (entropy ln perplexity), restarts E at 1; refinement then moves the
    lists to the new metric's neighbours; switching back restores the
    Euclidean distances."""
    from scipy.spatial.distance import cdist
    O = oracle_lib
    X, _ = _rescaled_blobs(4, 50, 8, 12)
    N, K, perp = X.shape[0], 12, 5.0
    S = O.OracleState(X, 2, K, 8, 5, y_init(N, 2))
    hp = O.Hyper(perplexity=perp, lr=N / 12, attr=4.0, n_neg=4, hd_mode=1)
    S.init(hp)
    for _ in range(30):
        S.step(hp)
    before = S.hd_idx[:N].copy()
    S.E[0] = 0.25
    S.flags[:N] = 0
    S.set_metric(hp, 1)
    X64 = X.astype(np.float64)
    A = 2.0 * cdist(X64, X64, "cosine")
    for i in range(N):
        idx, d2 = S.hd_idx[i], S.hd_d2[i]
        assert set(idx) == set(before[i])
        np.testing.assert_allclose(d2, A[i, idx], rtol=1e-12, atol=1e-15)
        keys = list(zip(d2, idx))
        assert keys == sorted(keys)
        p = np.exp(-S.beta[i] * (d2 - S.m[i]))
        p /= p.sum()
        H = -np.sum(p[p > 0] * np.log(p[p > 0]))
        assert abs(H - np.log(perp)) < 1e-8
    assert np.all(S.flags[:N] == 1) and S.E[0] == 1.0
    assert 0.0 < S.P[:N].sum() <= 1.0 + 1e-12
    for _ in range(150):
        S.step(hp)
    np.fill_diagonal(A, np.inf)
    ex = np.argsort(A, axis=1, kind="stable")[:, :K]
    rec = np.mean([len(set(a) & set(b)) for a, b in zip(S.hd_idx[:N], ex)]) / K
    assert rec > 0.97, rec
    S.set_metric(hp, 0)
    for i in range(0, N, 5):
        np.testing.assert_allclose(S.hd_d2[i], ((X64[S.hd_idx[i]] - X64[i]) ** 2).sum(1),
                                   rtol=1e-12)


# --- renumbering (a relabelling of the state, for memory locality) ----------
def test_renumber_relabels_the_state(oracle_lib):
    """The identity changes nothing; a permutation and its inverse restore the
    state exactly; every stored distance is the distance between the
    renumbered rows and every list holds the mapped set of points."""
    O = oracle_lib
    X, _ = blobs(n_clusters=4, per_cluster=50, D=8, seed=31)
    N, K = X.shape[0], 12
    S = O.OracleState(X, 2, K, 8, 5, y_init(N, 2))
    hp = O.Hyper(perplexity=5.0, lr=N / 12, attr=4.0, n_neg=4, hd_mode=1)
    S.init(hp)
    for _ in range(10):
        S.step(hp)
    ref = S.copy()
    names = ("X", "Y", "V", "hd_idx", "hd_d2", "ld_idx", "beta", "m", "r", "invS", "P", "flags")
    S.renumber(np.arange(N))
    for k in names:
        assert np.array_equal(S.live(k), ref.live(k)), k
    p = np.random.default_rng(4).permutation(N)
    S.renumber(p)
    Xd = S.live("X").astype(np.float64)
    for i_old in range(0, N, 9):
        i = p[i_old]
        assert set(S.hd_idx[i].tolist()) == set(p[ref.hd_idx[i_old]].tolist())
        np.testing.assert_allclose(S.hd_d2[i], ((Xd[S.hd_idx[i]] - Xd[i]) ** 2).sum(1),
                                   rtol=1e-12)
        assert np.array_equal(S.Y[i], ref.Y[i_old]) and np.array_equal(S.P[i], ref.P[i_old])
    inv = np.empty(N, dtype=np.int64)
    inv[p] = np.arange(N)
    S.renumber(inv)
    for k in names:
        assert np.array_equal(S.live(k), ref.live(k)), k
    with pytest.raises(ValueError):
        S.renumber(np.zeros(N, dtype=np.int64))
