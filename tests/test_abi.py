"""The C ABI: every symbol declared in include/fsne.h is exported by
libfsne.so, and argument checking rejects bad calls before any device work
(so these run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(fsne_\w+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("fsne_init", "fsne_step", "fsne_set_hyperparams", "fsne_get_Y", "fsne_get_knn",
              "fsne_get_state", "fsne_set_state", "fsne_destroy", "fsne_insert_points",
              "fsne_drift_points"):
        assert n in names


def test_library_exports_every_declared_symbol(fsne_lib):
    lib = C.CDLL(fsne_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_defaults_and_argument_checks(fsne_lib):
    F = fsne_lib
    hp = F.fsne_default_hparams()
    assert hp.alpha == 1.0 and hp.p_min == np.float32(0.05) and hp.hd_mode == 0
    assert hp.reject_memo == 1 and hp.metric == 0
    L = F.load_library()
    assert L.fsne_default_hparams(None) == F.FSNE_EINVAL
    X = np.zeros((100, 8), np.float32)
    ctx = C.c_void_p()

    def init(**kw):
        a = dict(X=X.ctypes.data, N=100, D=8, xdt=0, Y0=None, d=2, Kh=16, Kl=8, alpha=1.0,
                 perp=10.0, seed=1, hp=None, dev=0, stream=None, cap=100)
        a.update(kw)
        return L.fsne_init(C.byref(ctx), a["X"], a["N"], a["D"], a["xdt"], a["Y0"], a["d"],
                           a["Kh"], a["Kl"], a["alpha"], a["perp"], a["seed"], a["hp"], a["dev"],
                           a["stream"], a["cap"])

    assert init(Kh=100) == F.FSNE_EINVAL          # K_hd >= N
    X300 = np.zeros((300, 8), np.float32)
    assert init(X=X300.ctypes.data, N=300, cap=300, Kh=257) == F.FSNE_EINVAL   # K_hd <= 256
    assert init(Kl=65) == F.FSNE_EINVAL           # LD list longer than a wave
    assert init(Kh=1) == F.FSNE_EINVAL
    assert init(Kl=0) == F.FSNE_EINVAL
    assert init(d=0) == F.FSNE_EINVAL
    assert init(d=65) == F.FSNE_EINVAL
    assert init(xdt=7) == F.FSNE_EINVAL
    assert init(X=None) == F.FSNE_EINVAL
    assert init(cap=50) == F.FSNE_EINVAL
    # widest rows: FP32 4096 (D % 4 == 0), BF16 2048 (D % 8 == 0), else 1024
    assert L.fsne_max_dim(0, 4096) == 4096 and L.fsne_max_dim(0, 1023) == 1024
    assert L.fsne_max_dim(1, 2048) == 2048 and L.fsne_max_dim(1, 1020) == 1024
    assert init(D=4100) == F.FSNE_EINVAL
    assert init(D=1025) == F.FSNE_EINVAL
    assert init(D=2056, xdt=1) == F.FSNE_EINVAL
    # alpha and perplexity are positional and replace the hyperparameters' values
    assert init(alpha=0.0) == F.FSNE_EINVAL
    assert init(alpha=-1.0) == F.FSNE_EINVAL
    assert init(perp=16.0) == F.FSNE_EINVAL        # >= K_hd: no finite calibration
    assert init(perp=1.0) == F.FSNE_EINVAL
    for bad in (dict(momentum=1.0), dict(n_neg=65), dict(hd_mode=3), dict(dist_mode=1),
                dict(e_smooth=0.0), dict(lr=float("nan")), dict(reject_memo=2),
                dict(reject_memo=-1), dict(metric=2), dict(metric=-1)):
        h = F.fsne_default_hparams(**bad)
        assert init(hp=C.byref(h)) == F.FSNE_EINVAL, bad
    assert not ctx.value
    # null contexts are rejected, destroy(NULL) is a no-op
    assert L.fsne_step(None, 1) == F.FSNE_EINVAL
    assert L.fsne_sync(None) == F.FSNE_EINVAL
    L.fsne_destroy(None)
    assert L.fsne_last_error(None) == b"null context"


def test_hierarchy_edges_worked_example(fsne_lib):
    """Host-only entry point: overlap of clusters over the smaller size.
    Level g: A0 = {0,1,2,3}, A1 = {4,5}; level h: B0 = {0,1}, B1 = {2,3,4},
    B2 = {5}; point 6 is noise at both levels.  By hand:
      E[A0,B0] = 2/2, E[A0,B1] = 2/3, E[A0,B2] = 0/1,
      E[A1,B0] = 0/2, E[A1,B1] = 1/2, E[A1,B2] = 1/1."""
    F = fsne_lib
    la = [0, 0, 0, 0, 1, 1, -1]
    lb = [0, 0, 1, 1, 1, 2, -1]
    E = F.fsne_hierarchy_edges(la, 2, lb, 3)
    want = np.array([[1.0, 2 / 3, 0.0], [0.0, 0.5, 1.0]], dtype=np.float32)
    np.testing.assert_allclose(E, want, rtol=1e-7)
