"""The one-point oracle step against the whole-step oracle.

`fsneo_point_step` recomputes one point's iteration from the state before it
(refining the point and the members of its new HD list, recalibrating those
that changed, then its affinities and its LD phase).  It is the checker of
every full-size parity case, so it is pinned here to `fsneo_step`, the
whole-method step it must agree with: for every point of small states, with
the HD refinement on and off, under both HD metrics and on a renumbered
state, every output must equal what the full step writes for that point,
bit for bit (both are the same double-precision arithmetic).  Builds of the
oracle with a planted mistake in the one-point path (a neighbour's stale
record, stale neighbour rows in the LD phase, a stale membership test, the
point's own stale record) must fail it.
"""
import os

import numpy as np
import pytest

from inputs.generators import blobs, manifolds, y_init

CASES = {
    "blobs_600": lambda: (blobs(n_clusters=6, per_cluster=100, D=10, seed=31)[0],
                          dict(d=2, K_hd=16, K_ld=8, n_neg=5, alpha=1.0, perplexity=6.0)),
    "manifold_700": lambda: (manifolds(n_manifolds=7, per_manifold=100, D=24, k=3, seed=32)[0],
                             dict(d=5, K_hd=12, K_ld=10, n_neg=4, alpha=0.6, perplexity=5.0)),
}


def _hp(O, N, c, hd_mode):
    return O.Hyper(alpha=c["alpha"], perplexity=c["perplexity"], lr=N / 12.0, momentum=0.5,
                   attr=12.0, rep=1.0, n_neg=c["n_neg"], hd_mode=hd_mode, e_smooth=0.1,
                   p_min=0.05)


def _state(O, name, metric=0, renumber=False, warm=2):
    X, c = CASES[name]()
    N = X.shape[0]
    S = O.OracleState(X, c["d"], c["K_hd"], c["K_ld"], 42, y_init(N, c["d"]),
                      metric=metric).init(_hp(O, N, c, 1))
    for it in range(warm):
        S.step(_hp(O, N, c, 1 if it % 2 == 0 else 0))
    if renumber:
        S.renumber(np.random.default_rng(5).permutation(N))
    return S, c


def _mismatches(O, S0, c, fired, limit=None):
    """Points whose one-point recomputation differs from the full step."""
    N = S0.N
    hp = _hp(O, N, c, 1 if fired else 2)
    S1 = S0.copy()
    out = S1.step(hp, want_partials=True)
    assert out["fired"] == fired
    bad = []
    for i in range(N if limit is None else limit):
        ps = S0.point_step(hp, i, fired)
        rec = np.array([S1.beta[i], S1.m[i], S1.r[i], S1.invS[i]])
        same = (np.array_equal(ps["hd_idx"], S1.hd_idx[i])
                and np.array_equal(ps["hd_d2"], S1.hd_d2[i])
                and np.array_equal(ps["rec"], rec)
                and np.array_equal(ps["P"], S1.P[i])
                and np.array_equal(ps["ld_idx"], S1.ld_idx[i])
                and np.array_equal(ps["A"], out["A"][i])
                and np.array_equal(ps["R"], out["R"][i])
                and ps["Zh"] == out["Zh"][i])
        if fired:
            same = same and ps["flag"] == S1.flags[i]
        if not same:
            bad.append(i)
    return bad


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("metric,renumber", [(0, False), (1, False), (0, True)])
@pytest.mark.parametrize("fired", [1, 0])
def test_point_step_equals_full_step(oracle_lib, name, metric, renumber, fired):
    O = oracle_lib
    S0, c = _state(O, name, metric=metric, renumber=renumber)
    bad = _mismatches(O, S0, c, fired)
    assert not bad, f"{len(bad)} points differ, first {bad[:8]}"


def test_point_step_equals_full_step_later(oracle_lib):
    """After some iterations (fewer lists change per refinement)."""
    O = oracle_lib
    S0, c = _state(O, "blobs_600", warm=25)
    assert _mismatches(O, S0, c, 1) == []


@pytest.mark.parametrize("plant", [1, 2, 3, 4])
def test_planted_mistakes_are_caught(oracle_lib, tmp_path, plant):
    O = oracle_lib
    path = O.build_oracle(path=os.path.join(str(tmp_path), f"liboracle_plant{plant}.so"),
                          defines=(f"FSNEO_PLANT={plant}",))
    with O.using_library(path):
        S0, c = _state(O, "blobs_600")
        bad = _mismatches(O, S0, c, 1, limit=200)
    assert len(bad) > 0, f"planted mistake {plant} went unnoticed"
