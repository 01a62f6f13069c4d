"""Error paths of the library on the GPU, forced from the host.

Every kernel still runs to completion: the calls return the documented
status, change nothing they reject, and leave the context usable.
"""
import numpy as np
import pytest

from inputs.generators import blobs, y_init

pytestmark = [pytest.mark.gpu]


def _emb(F, N=600, capacity=None):
    X, _ = blobs(n_clusters=4, per_cluster=N // 4, D=16, seed=3)
    hp = F.fsne_default_hparams(perplexity=8.0, lr=N / 12.0, n_neg=8)
    return X, F.Embedding(X, y_init(N, 2), 2, 16, 8, seed=2, hp=hp, capacity=capacity)


def test_insert_beyond_capacity(fsne_lib):
    F = fsne_lib
    X, emb = _emb(F, capacity=650)
    emb.step(3)
    Xn = X[:100] + np.float32(0.01)
    with pytest.raises(F.FsneError) as e:
        emb.insert(Xn)                       # 600 + 100 > 650
    assert e.value.status == F.FSNE_ENOMEM
    assert emb.stats()["N"] == 600
    emb.insert(Xn[:50])                      # fills the capacity exactly
    assert emb.stats()["N"] == 650 and emb.N == 650
    emb.step(3)
    st = emb.stats()
    assert st["N"] == 650 and st["nonfinite"] == 0
    idx, _ = emb.knn(0)
    assert idx.shape == (650, 16) and np.all((idx >= 0) & (idx < 650))
    emb.close()


def test_delete_rejects_bad_ids(fsne_lib):
    F = fsne_lib
    X, emb = _emb(F, capacity=600)
    emb.step(2)
    snap = emb.state(["Y", "hd_idx", "ld_idx"])
    for bad in ([600], [-1], [3, 7, 3], list(range(590))):   # range, sign, duplicate, too many
        with pytest.raises(F.FsneError) as e:
            emb.delete(np.array(bad, dtype=np.int64))
        assert e.value.status == F.FSNE_EINVAL, bad
        assert emb.stats()["N"] == 600
    after = emb.state(["Y", "hd_idx", "ld_idx"])
    for k in snap:
        np.testing.assert_array_equal(after[k], snap[k])
    emb.delete(np.array([], dtype=np.int64))                 # nothing to do
    emb.delete(np.array([0, 599, 300], dtype=np.int64))
    assert emb.stats()["N"] == 597 and emb.N == 597
    emb.step(2)
    assert emb.stats()["nonfinite"] == 0
    emb.close()


def test_nonfinite_embedding_is_reported(fsne_lib):
    F = fsne_lib
    _, emb = _emb(F)
    emb.step(2)
    Y = emb.Y()
    bad = Y.copy()
    bad[5, 0] = np.nan
    emb.set_state({"Y": bad})
    emb.step(1)
    st = emb.stats()
    assert st["nonfinite"] == 1 and st["status"] == F.FSNE_ENONFINITE
    # a finite state clears the report
    emb.set_state({"Y": Y, "V": np.zeros_like(Y)})
    emb.step(2)
    st = emb.stats()
    assert st["nonfinite"] == 0 and st["status"] == F.FSNE_OK
    assert np.all(np.isfinite(emb.Y()))
    emb.close()


def test_invalid_arguments_leave_the_context_unchanged(fsne_lib):
    F = fsne_lib
    _, emb = _emb(F)
    emb.step(2)
    before = emb.hyperparams().as_dict()
    for kw in (dict(alpha=-1.0), dict(perplexity=20.0), dict(momentum=1.5), dict(n_neg=65)):
        with pytest.raises(F.FsneError) as e:
            emb.set_hyperparams(F.fsne_default_hparams(**{**before, **kw}))
        assert e.value.status == F.FSNE_EINVAL, kw
        assert emb.hyperparams().as_dict() == before
    with pytest.raises(F.FsneError) as e:
        emb.step(-1)
    assert e.value.status == F.FSNE_EINVAL
    t = emb.stats()["t"]
    emb.step(0)
    assert emb.stats()["t"] == t
    emb.step(1)
    assert emb.stats()["t"] == t + 1
    emb.close()
