"""Affinities kept up to date over many refinements.

A refinement recomputes the affinity of a list entry only when one of its
two points changed its list; every other entry keeps its value.  After many
iterations without any injected state the kept values must equal (1) a full
recomputation from the same lists and records (state set again without P,
which recomputes every entry) bit for bit, and (2) eq. (1) restricted to the
lists, evaluated here from those lists and records:
    p_ij = (p_{j|i} + [i in list(j)] p_{i|j}) / 2N,
    p_{j|i} = exp(-beta_i (d2_ij - m_i)) / S_i.
"""
import numpy as np
import pytest

from inputs.generators import f32_to_bf16_bits, manifolds, y_init, zipf_mixture

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

CASES = {
    "manifold_2500_K32": (lambda: manifolds(per_manifold=50, seed=1003)[0][:2500], 16, 32, 32),
    "zipf_2100_bf16_K64": (lambda: f32_to_bf16_bits(zipf_mixture(N=2100, n_clusters=20,
                                                                 seed=1005)[0]), 32, 64, 32),
}


def _eq1_restricted(hd_idx, hd_d2, rec):
    N, K = hd_idx.shape
    beta, m, invS = (rec[:, 0].astype(np.float64), rec[:, 1].astype(np.float64),
                     rec[:, 3].astype(np.float64))
    d2 = hd_d2.astype(np.float64)
    pji = np.exp(-beta[:, None] * (d2 - m[:, None])) * invS[:, None]
    j = hd_idx
    member = np.zeros((N, K), dtype=bool)
    rows = np.arange(N)
    for k in range(K):
        member[:, k] = np.any(hd_idx[j[:, k]] == rows[:, None], axis=1)
    pij = np.where(member, np.exp(-beta[j] * (d2 - m[j])) * invS[j], 0.0)
    return (pji + pij) / (2.0 * N)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("hd_mode", [1, 0])
def test_kept_affinities_equal_full_recomputation(fsne_lib, case, hd_mode):
    F = fsne_lib
    make, d, Kh, Kl = CASES[case]
    X = make()
    N = X.shape[0]
    hp = F.fsne_default_hparams(alpha=1.0, perplexity=10.0, lr=N / 12.0, n_neg=16,
                                hd_mode=hd_mode)
    emb = F.Embedding(X, y_init(N, d), d, Kh, Kl, seed=5, hp=hp)
    emb.step(60)
    st = emb.stats()
    assert st["nonfinite"] == 0
    g = emb.state(["hd_idx", "hd_d2", "rec", "P", "flags"])
    # some refinements changed only part of the lists, so entries were kept
    assert 0 < st["E"] < 1
    emb.set_state({"hd_idx": g["hd_idx"], "hd_d2": g["hd_d2"], "rec": g["rec"]})
    full = emb.state(["P"])["P"]
    np.testing.assert_array_equal(g["P"], full)
    ref = _eq1_restricted(g["hd_idx"], g["hd_d2"], g["rec"])
    err = np.abs(g["P"].astype(np.float64) - ref)
    assert np.all(err <= 1e-5 * ref + 1e-12 / N), float(np.max(err / np.maximum(ref, 1e-30)))
    emb.close()
