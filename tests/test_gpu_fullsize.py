"""Full-size checks of the step, in the benchmark's launch configuration.

At the workloads' real sizes the whole-step oracle is too slow, so sampled
points (random ones plus the first and the last, which sits in the ragged
tail of the grid) are recomputed one by one.  Two starting states:

* the oracle's own initial state, injected into the GPU (random lists: every
  point changes);
* a steady state: the GPU runs 300 iterations of the benchmark's schedule
  (renumbered every 25 up to iteration 275, then 25 refining iterations with
  the memory of rejected candidates filling), its state is read and loaded
  into the oracle, and the GPU takes one more refining step from it (with
  its memory and its incrementally updated affinities).

For each sampled point i the GPU's step is checked phase by phase against
the oracle run on the same inputs:
* HD row: `fsneo_hd_refine_point` from the state before the step; rows equal
  or differing only at FP32 ties (the BF16 screen may also have dropped a
  candidate that would have entered: a valid row whose last distance is not
  smaller, counted separately); flag equal;
* calibration of i and of every member of its new list: the oracle
  calibrates the GPU's rows of the flagged ones, the others keep their
  records;
* P row of i: `fsneo_psym_row` on the GPU's new lists with those records;
* LD phase of i: `fsneo_ld_refine_grad_point` on the GPU's new HD lists and
  P: LD row by the LD tie rule, A, R, Zh;
and by `fsneo_point_step`, the oracle's whole step for one point (pinned to
the whole-step oracle on the CPU), where i's and its neighbours' inputs agree
(rows differing at ties excused with their reason checked).

Under the angular HD metric the distances carry the FP32 row-scale error
bounded in tests/test_gpu_metric.py (4 eps sqrt(d2) more, eps = (D/2 + 3) u),
and the affinities and partials are compared within 1e-3 instead of 1e-4.
"""
import numpy as np
import pytest

from inputs.generators import f32_to_bf16_bits, make_workload, y_init
from tests.parity import exact_d2, hd_tie_tol, ld_tie_tol, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

# name: (workload, BF16 rows, dist_mode, alpha override, HD metric, renumbered, steady)
CASES = {
    "image_70k_f32": ("image_70k", False, 0, 1.0, 0, False, False),
    "image_70k_f32_a05": ("image_70k", False, 0, 0.5, 0, False, False),
    "image_70k_f32_a4": ("image_70k", False, 0, 4.0, 0, False, False),
    "manifold_1m_f32": ("manifold_1m", False, 0, None, 0, False, False),
    # the benchmark's configuration: the state renumbered (fsne_reorder) on the
    # GPU and the same permutation applied to the oracle's state
    "manifold_1m_f32_renumbered": ("manifold_1m", False, 0, None, 0, True, False),
    "manifold_1m_f32_angular": ("manifold_1m", False, 0, None, 1, False, False),
    "manifold_1m_bf16_screen": ("manifold_1m", True, 1, None, 0, False, False),
    "zipf_4m_bf16": ("zipf_4m", True, 0, None, 0, False, False),
    "zipf_4m_bf16_screen": ("zipf_4m", True, 1, None, 0, False, False),
    # steady state after 300 GPU iterations (renumbered, remembered rejections,
    # affinities updated incrementally), the benchmarked FP32 and BF16 forms
    "manifold_1m_f32_steady": ("manifold_1m", False, 0, None, 0, True, True),
    "manifold_1m_bf16_screen_steady": ("manifold_1m", True, 1, None, 0, True, True),
}

U = 2.0 ** -24
N_SAMPLES = 64


def _exact_d2(X, i, ids, metric):
    if metric == 0:
        return exact_d2(X, i, ids)
    from inputs.generators import bf16_bits_to_f32
    Xf = bf16_bits_to_f32(X) if X.dtype == np.uint16 else X
    rows = Xf[np.concatenate([[i], np.asarray(ids)])].astype(np.float64)
    n = np.sqrt((rows * rows).sum(1, keepdims=True))
    rows = np.where(n > 0, rows / np.where(n > 0, n, 1.0), 0.0)
    return ((rows[1:] - rows[0]) ** 2).sum(1)


def _d2_bound(D, bf16, metric, d2):
    """|GPU d2 - exact d2| allowed for one entry."""
    tol = hd_tie_tol(D, bf16)
    if metric == 0:
        return 0.5 * tol * d2
    eps = (D / 2 + 3) * U
    return 4.0 * eps * np.sqrt(np.maximum(d2, 0.0)) + 0.5 * tol * d2


def _schedule(F, hp, t):
    """The benchmark's schedule: exaggeration 12 and momentum 0.5 for 250
    iterations, then 1 and 0.8."""
    late = t >= 250
    return F.fsne_default_hparams(**{**hp.as_dict(), "attr": 1.0 if late else 12.0,
                                     "momentum": 0.8 if late else 0.5})


@pytest.mark.parametrize("case", list(CASES))
def test_fullsize_sampled_step(oracle_lib, fsne_lib, case):
    O, F = oracle_lib, fsne_lib
    name, bf16, dist_mode, alpha_override, metric, renumbered, steady = CASES[case]
    print(f"case {case}", flush=True)
    X, _, cfg = make_workload(name)
    if bf16:
        X = f32_to_bf16_bits(X)
    N, D = X.shape
    K, Kl, d = cfg["K_hd"], cfg["K_ld"], cfg["d"]
    alpha = alpha_override if alpha_override is not None else cfg["alpha"]
    kw = dict(alpha=alpha, perplexity=cfg["perplexity"], lr=float(np.float32(N / 12.0)),
              momentum=0.5, attr=12.0, rep=1.0, n_neg=cfg["n_neg"], hd_mode=1, e_smooth=0.1,
              p_min=0.05)
    hp_g = F.fsne_default_hparams(**kw, dist_mode=dist_mode, metric=metric)
    Y0 = y_init(N, d)
    emb = F.Embedding(X, Y0, d, K, Kl, seed=42, hp=hp_g)
    if steady:
        # 275 iterations under the coin with the schedule, renumbered every 25;
        # then 25 refining iterations without renumbering, so that the memory
        # of rejected candidates fills (a renumbering clears it)
        hp_c = F.fsne_default_hparams(**{**hp_g.as_dict(), "hd_mode": 0})
        for t0 in range(0, 275, 25):
            emb.set_hyperparams(_schedule(F, hp_c, t0))
            emb.step(25)
            p = emb.reorder()
            X = X[np.argsort(p)]           # row k of the renumbered X
        hp_g = F.fsne_default_hparams(**{**_schedule(F, hp_c, 275).as_dict(), "hd_mode": 1})
        emb.set_hyperparams(hp_g)
        emb.step(25)
        assert emb.stats()["nonfinite"] == 0
        g0 = emb.state()
        S = O.OracleState.from_gpu_state(X, g0, d, K, Kl, 42, metric=metric)
    else:
        S = O.OracleState(X, d, K, Kl, 42, Y0, metric=metric).init(O.Hyper(**kw))
        S.round_to_f32()
        emb.set_state(S.as_gpu_state())
        if renumbered:
            p = emb.reorder()
            assert np.array_equal(np.sort(p), np.arange(N))
            S.renumber(p)
            X = S.live("X")
    hpd = hp_g.as_dict()
    hp_o = O.Hyper(alpha=float(np.float32(hpd["alpha"])),
                   perplexity=float(np.float32(hpd["perplexity"])),
                   lr=float(np.float32(hpd["lr"])), momentum=float(np.float32(hpd["momentum"])),
                   attr=float(np.float32(hpd["attr"])), rep=1.0, n_neg=cfg["n_neg"], hd_mode=1,
                   e_smooth=float(np.float32(0.1)), p_min=float(np.float32(0.05)))
    emb.step(1)
    g = emb.state(["hd_idx", "hd_d2", "ld_idx", "rec", "P", "flags", "A", "R", "Zh"])
    st = emb.stats()
    assert st["last_fired"] == 1 and st["nonfinite"] == 0
    rng = np.random.default_rng(17)
    samples = np.unique(np.concatenate([[0, N - 1], rng.choice(N, N_SAMPLES - 2, replace=False)]))
    rtol_fp = 1e-4 if metric == 0 else 1e-3
    gflag = g["flags"] & 1
    grec = g["rec"].astype(np.float64)
    # the oracle's view of the state after the GPU's HD phase
    post = S.copy()
    post.hd_idx[:N] = g["hd_idx"]
    post.hd_d2[:N] = g["hd_d2"]
    post.beta[:N], post.m[:N], post.r[:N], post.invS[:N] = grec.T
    Pg = g["P"].astype(np.float64)
    Yf = S.live("Y")
    ld_tol = ld_tie_tol(d)
    hd_ties = screened = ld_ties = excused = 0
    for i in samples:
        i = int(i)
        # HD row of i from the state before the step
        oi, od, oflag = S.hd_refine_point(i)
        gi = g["hd_idx"][i]
        if np.array_equal(gi, oi):
            assert gflag[i] == oflag, (case, i)
            assert np.all(np.abs(g["hd_d2"][i] - od) <=
                          2.0 * _d2_bound(D, bf16, metric, od) + 1e-30), (case, i)
        else:
            dg = _exact_d2(X, i, gi, metric)
            assert len(set(gi.tolist())) == K and i not in set(gi.tolist()), (case, i)
            if np.all(np.abs(dg - od) <= 2.0 * _d2_bound(D, bf16, metric, od) + 1e-30):
                hd_ties += 1
            else:
                assert dist_mode == 1 and dg[-1] >= od[-1] * (1 - 1e-6), (case, i)
                screened += 1
        # calibration of i and of the members of its new list
        for j in [i, *gi.tolist()]:
            if gflag[j]:
                rec, _ = O.calibrate(g["hd_d2"][j].astype(np.float64), hp_o.perplexity)
                assert abs(grec[j, 0] - rec[0]) <= rtol_fp * rec[0], (case, i, j)
                assert abs(grec[j, 3] - rec[3]) <= rtol_fp * rec[3], (case, i, j)
                post.beta[j], post.m[j], post.r[j], post.invS[j] = rec
            else:
                kept = np.array([S.beta[j], S.m[j], S.r[j], S.invS[j]], np.float32)
                assert np.array_equal(grec[j], kept), (case, j)
        # affinities of i from the GPU's new lists
        assert rel_l2(g["P"][i], post.psym_row(i)) < rtol_fp, (case, i)
        # LD phase of i from the GPU's new HD lists and P
        ld, A, R, Zh = S.ld_refine_grad_point(hp_o, i, hd_next=g["hd_idx"], P_next=Pg)
        assert rel_l2(g["A"][i], A) < rtol_fp, (case, i)
        if np.array_equal(g["ld_idx"][i], ld):
            assert rel_l2(g["R"][i], R) < rtol_fp, (case, i)
            assert abs(g["Zh"][i] - Zh) <= 1e-5 * Zh, (case, i)
        else:
            gl = g["ld_idx"][i]
            assert len(set(gl.tolist())) == Kl and i not in set(gl.tolist()), (case, i)
            dgl = ((Yf[gl] - Yf[i]) ** 2).sum(1)
            dol = ((Yf[ld] - Yf[i]) ** 2).sum(1)
            assert np.all(np.abs(dgl - dol) <= ld_tol * dol), (case, i)
            ld_ties += 1
        # the oracle's whole step for i where its inputs agree exactly
        o = S.point_step(hp_o, i, 1)
        nb = o["hd_idx"]
        if not (np.array_equal(g["hd_idx"][i], nb)
                and all(np.array_equal(g["hd_idx"][j], S.hd_refine_point(int(j))[0])
                        for j in nb)):
            excused += 1          # i's or a neighbour's row differs at a tie (checked above)
            continue
        assert rel_l2(g["P"][i], o["P"]) < rtol_fp, (case, i)
        if np.array_equal(g["ld_idx"][i], o["ld_idx"]):
            assert rel_l2(g["A"][i], o["A"]) < rtol_fp, (case, i)
            assert rel_l2(g["R"][i], o["R"]) < rtol_fp, (case, i)
    print(f"{case}: {len(samples)} samples, HD ties {hd_ties}, lost to the screen {screened}, "
          f"LD ties {ld_ties}, whole-step comparisons excused {excused}", flush=True)
    assert hd_ties + ld_ties <= 3 and screened <= 3, (case, hd_ties, ld_ties, screened)
    # properties of the whole state
    hd = g["hd_idx"]
    assert np.all(np.diff(g["hd_d2"], axis=1) >= 0)
    assert np.all(hd >= 0) and np.all(hd < N) and np.all(g["ld_idx"] < N)
    assert not (hd == np.arange(N)[:, None]).any()
    emb.close()
