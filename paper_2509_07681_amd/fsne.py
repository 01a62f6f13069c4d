"""Python binding of libfsne.so: argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own.  There is no fallback: if the HIP library is missing
or the GPU is unavailable, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsne.so")

FSNE_OK, FSNE_EINVAL, FSNE_ENOMEM, FSNE_EHIP, FSNE_ESTATE, FSNE_ENONFINITE = 0, -1, -2, -3, -4, -5
FSNE_F32, FSNE_BF16 = 0, 1


class FsneError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fsne error {status}: {msg}")
        self.status = status


class fsne_hparams(C.Structure):
    _fields_ = [("alpha", C.c_float), ("perplexity", C.c_float), ("lr", C.c_float),
                ("momentum", C.c_float), ("attr", C.c_float), ("rep", C.c_float),
                ("n_neg", C.c_int32), ("hd_mode", C.c_int32), ("dist_mode", C.c_int32),
                ("e_smooth", C.c_float), ("p_min", C.c_float), ("rerank_margin", C.c_float),
                ("reject_memo", C.c_int32), ("metric", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fsne_state_view(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("Y", "V", "hd_idx", "hd_d2", "ld_idx", "rec", "P",
                                          "flags", "A", "R", "Zh", "E", "t")]


class fsne_stats(C.Structure):
    _fields_ = [("N", C.c_int64), ("t", C.c_uint32), ("E", C.c_float), ("next_fire", C.c_int32),
                ("last_fired", C.c_int32), ("n_new", C.c_int32), ("Z", C.c_float),
                ("nonfinite", C.c_int32), ("hd_cand_rows", C.c_uint32),
                ("ld_cand_rows", C.c_uint32), ("hd_refinements", C.c_uint32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfsne.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_2509_07681_amd/build.py")
    L = C.CDLL(path)
    P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    L.fsne_default_hparams.argtypes = [C.POINTER(fsne_hparams)]
    L.fsne_init.argtypes = [C.POINTER(P), P, I64, I32, I32, P, I32, I32, I32, F, F,
                            C.c_uint64, C.POINTER(fsne_hparams), I32, P, I64]
    L.fsne_step.argtypes = [P, I32]
    L.fsne_set_hyperparams.argtypes = [P, C.POINTER(fsne_hparams)]
    L.fsne_get_hyperparams.argtypes = [P, C.POINTER(fsne_hparams)]
    L.fsne_get_Y.argtypes = [P, P, I32]
    L.fsne_get_knn.argtypes = [P, I32, P, P]
    L.fsne_get_state.argtypes = [P, C.POINTER(fsne_state_view)]
    L.fsne_set_state.argtypes = [P, C.POINTER(fsne_state_view)]
    L.fsne_get_stats.argtypes = [P, C.POINTER(fsne_stats)]
    L.fsne_sync.argtypes = [P]
    L.fsne_insert_points.argtypes = [P, P, I64, P]
    L.fsne_drift_points.argtypes = [P, P, P, I64, P]
    L.fsne_drift_points_noalloc.argtypes = [P, P, P, I64, P]
    L.fsne_implode.argtypes = [P, F]
    L.fsne_jump_start.argtypes = [P, I32, F]
    L.fsne_delete_points.argtypes = [P, P, I64]
    L.fsne_renumber.argtypes = [P, P]
    L.fsne_reorder.argtypes = [P, P]
    L.fsne_reorder_data.argtypes = [P, P]
    L.fsne_cluster.argtypes = [P, F, I32, P, P]
    L.fsne_hierarchy_edges.argtypes = [P, I32, P, I32, I64, P]
    L.fsne_destroy.argtypes = [P]
    L.fsne_destroy.restype = None
    L.fsne_last_error.argtypes = [P]
    L.fsne_last_error.restype = C.c_char_p
    for name in ("fsne_default_hparams", "fsne_init", "fsne_step", "fsne_set_hyperparams",
                 "fsne_get_hyperparams", "fsne_get_Y", "fsne_get_knn", "fsne_get_state",
                 "fsne_set_state", "fsne_get_stats", "fsne_sync", "fsne_insert_points",
                 "fsne_drift_points", "fsne_drift_points_noalloc", "fsne_implode", "fsne_jump_start", "fsne_delete_points",
                 "fsne_cluster", "fsne_hierarchy_edges"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _check(ctx, st):
    if st != FSNE_OK:
        msg = load_library().fsne_last_error(ctx).decode() if ctx else "invalid argument"
        raise FsneError(st, msg)


def fsne_default_hparams(**overrides) -> fsne_hparams:
    hp = fsne_hparams()
    _check(None, load_library().fsne_default_hparams(C.byref(hp)))
    for k, v in overrides.items():
        if not hasattr(hp, k):
            raise AttributeError(k)
        setattr(hp, k, v)
    return hp


def fsne_init(X, Y0, d, K_hd, K_ld, seed, hp=None, stream=None, capacity=None, alpha=None,
              perplexity=None):
    """X: float32 array (host numpy or device torch tensor) or uint16 BF16 bits.
    alpha, perplexity: None takes them from hp (or the defaults)."""
    L = load_library()
    base = hp if hp is not None else fsne_default_hparams()
    alpha = base.alpha if alpha is None else alpha
    perplexity = base.perplexity if perplexity is None else perplexity
    on_dev = hasattr(X, "is_cuda") and X.is_cuda
    if on_dev:
        import torch

        if X.dtype == torch.float32:
            xdt = FSNE_F32
        elif X.dtype in (torch.bfloat16, torch.int16, torch.uint16):
            xdt = FSNE_BF16
        else:
            raise TypeError("X must be float32 or bfloat16")
        if not X.is_contiguous():
            raise ValueError("X must be contiguous")
        N, D = X.shape
    else:
        X = np.ascontiguousarray(X)
        if X.dtype == np.float32:
            xdt = FSNE_F32
        elif X.dtype == np.uint16:
            xdt = FSNE_BF16
        else:
            raise TypeError("X must be float32 or uint16 (BF16 bits)")
        N, D = X.shape
    Y0a = None if Y0 is None else np.ascontiguousarray(Y0, dtype=np.float32)
    if Y0a is not None and Y0a.shape != (N, d):
        raise ValueError("Y0 must be N x d")
    ctx = C.c_void_p()
    st = L.fsne_init(C.byref(ctx), _ptr(X), N, D, xdt, _ptr(Y0a), d, K_hd, K_ld, float(alpha),
                     float(perplexity), seed, C.byref(hp) if hp is not None else None,
                     1 if on_dev else 0,
                     None if stream is None else C.c_void_p(stream),
                     N if capacity is None else capacity)
    if st != FSNE_OK:
        raise FsneError(st, "fsne_init failed (invalid arguments or device error)")
    return ctx


def fsne_step(ctx, n_iters: int):
    _check(ctx, load_library().fsne_step(ctx, n_iters))


def fsne_set_hyperparams(ctx, hp: fsne_hparams):
    _check(ctx, load_library().fsne_set_hyperparams(ctx, C.byref(hp)))


def fsne_get_hyperparams(ctx) -> fsne_hparams:
    hp = fsne_hparams()
    _check(ctx, load_library().fsne_get_hyperparams(ctx, C.byref(hp)))
    return hp


def fsne_get_Y(ctx, N: int, d: int, out=None):
    on_dev = out is not None and hasattr(out, "is_cuda") and out.is_cuda
    if out is None:
        out = np.empty((N, d), dtype=np.float32)
    _check(ctx, load_library().fsne_get_Y(ctx, _ptr(out), 1 if on_dev else 0))
    return out


def fsne_get_knn(ctx, which: int, N: int, K: int, with_dist=True):
    idx = np.empty((N, K), dtype=np.int32)
    dist = np.empty((N, K), dtype=np.float32) if (with_dist and which == 0) else None
    _check(ctx, load_library().fsne_get_knn(ctx, which, _ptr(idx), _ptr(dist)))
    return idx, dist


_VIEW_SHAPES = {"Y": "Nd", "V": "Nd", "A": "Nd", "R": "Nd", "hd_idx": "Nh", "hd_d2": "Nh",
                "P": "Nh", "ld_idx": "Nl", "rec": "N4", "flags": "N", "Zh": "N"}
_VIEW_DTYPES = {"hd_idx": np.int32, "ld_idx": np.int32, "flags": np.uint8}


def fsne_get_state(ctx, N, d, K_hd, K_ld, fields=None):
    fields = fields or list(_VIEW_SHAPES) + ["E", "t"]
    dims = {"N": N, "d": d, "h": K_hd, "l": K_ld, "4": 4}
    out, view = {}, fsne_state_view()
    for f in fields:
        if f == "E":
            out[f] = np.zeros(1, np.float32)
        elif f == "t":
            out[f] = np.zeros(1, np.uint32)
        else:
            shp = tuple(dims[c] for c in _VIEW_SHAPES[f])
            out[f] = np.zeros(shp, dtype=_VIEW_DTYPES.get(f, np.float32))
        setattr(view, f, out[f].ctypes.data)
    _check(ctx, load_library().fsne_get_state(ctx, C.byref(view)))
    out = {k: (v[0] if k in ("E", "t") else v) for k, v in out.items()}
    return out


def fsne_set_state(ctx, state: dict):
    view = fsne_state_view()
    keep = []
    for f, v in state.items():
        if f in ("A", "R", "Zh"):
            continue
        if f == "E":
            a = np.array([v], dtype=np.float32)
        elif f == "t":
            a = np.array([v], dtype=np.uint32)
        else:
            a = np.ascontiguousarray(v, dtype=_VIEW_DTYPES.get(f, np.float32))
        keep.append(a)
        setattr(view, f, a.ctypes.data)
    _check(ctx, load_library().fsne_set_state(ctx, C.byref(view)))


def fsne_get_stats(ctx) -> dict:
    st = fsne_stats()
    rc = load_library().fsne_get_stats(ctx, C.byref(st))
    d = {k: getattr(st, k) for k, _ in st._fields_}
    if rc not in (FSNE_OK, FSNE_ENONFINITE):
        _check(ctx, rc)
    d["status"] = rc
    return d


def fsne_sync(ctx):
    _check(ctx, load_library().fsne_sync(ctx))


def fsne_insert_points(ctx, Xnew, Yinit=None):
    Xnew = np.ascontiguousarray(Xnew)
    Ya = None if Yinit is None else np.ascontiguousarray(Yinit, dtype=np.float32)
    _check(ctx, load_library().fsne_insert_points(ctx, _ptr(Xnew), Xnew.shape[0], _ptr(Ya)))


def fsne_drift_points(ctx, ids, Xnew, Yinit=None):
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    Xnew = np.ascontiguousarray(Xnew)
    Ya = None if Yinit is None else np.ascontiguousarray(Yinit, dtype=np.float32)
    _check(ctx, load_library().fsne_drift_points(ctx, _ptr(ids), _ptr(Xnew), ids.size, _ptr(Ya)))


def fsne_drift_points_noalloc(ctx, ids, Xnew, Yinit=None):
    """fsne_drift_points staged in the library's fixed device array (no device
    allocation); ids strictly increasing."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    Xnew = np.ascontiguousarray(Xnew)
    Ya = None if Yinit is None else np.ascontiguousarray(Yinit, dtype=np.float32)
    _check(ctx, load_library().fsne_drift_points_noalloc(ctx, _ptr(ids), _ptr(Xnew), ids.size,
                                                         _ptr(Ya)))


def fsne_implode(ctx, factor: float):
    _check(ctx, load_library().fsne_implode(ctx, float(factor)))


def fsne_delete_points(ctx, ids):
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    _check(ctx, load_library().fsne_delete_points(ctx, _ptr(ids), ids.size))


def fsne_renumber(ctx, new_of_old):
    p = np.ascontiguousarray(new_of_old, dtype=np.int32)
    _check(ctx, load_library().fsne_renumber(ctx, _ptr(p)))


def fsne_reorder(ctx, N):
    p = np.empty(N, dtype=np.int32)
    _check(ctx, load_library().fsne_reorder(ctx, _ptr(p)))
    return p


def fsne_reorder_data(ctx, N):
    p = np.empty(N, dtype=np.int32)
    _check(ctx, load_library().fsne_reorder_data(ctx, _ptr(p)))
    return p


def fsne_cluster(ctx, N, eps: float, min_pts: int):
    labels = np.empty(N, dtype=np.int32)
    nc = np.zeros(1, dtype=np.int32)
    _check(ctx, load_library().fsne_cluster(ctx, float(eps), int(min_pts), _ptr(labels), _ptr(nc)))
    return labels, int(nc[0])


def fsne_hierarchy_edges(la, ca: int, lb, cb: int):
    la = np.ascontiguousarray(la, dtype=np.int32)
    lb = np.ascontiguousarray(lb, dtype=np.int32)
    E = np.zeros((ca, cb), dtype=np.float32)
    st = load_library().fsne_hierarchy_edges(_ptr(la), int(ca), _ptr(lb), int(cb), la.size, _ptr(E))
    if st != FSNE_OK:
        raise FsneError(st, "fsne_hierarchy_edges: bad arguments")
    return E


def fsne_jump_start(ctx, projection: int, sigma: float):
    _check(ctx, load_library().fsne_jump_start(ctx, int(projection), float(sigma)))


def fsne_destroy(ctx):
    if ctx:
        load_library().fsne_destroy(ctx)


class Embedding:
    """Small owner of one context (destroys it on close / garbage collection)."""

    def __init__(self, X, Y0, d, K_hd, K_ld, seed=42, hp=None, stream=None, capacity=None):
        self.N = X.shape[0]
        self.d, self.K_hd, self.K_ld = d, K_hd, K_ld
        self.ctx = fsne_init(X, Y0, d, K_hd, K_ld, seed, hp, stream, capacity)

    def step(self, n=1):
        fsne_step(self.ctx, n)

    def set_hyperparams(self, hp):
        fsne_set_hyperparams(self.ctx, hp)

    def hyperparams(self):
        return fsne_get_hyperparams(self.ctx)

    def Y(self):
        return fsne_get_Y(self.ctx, self.N, self.d)

    def knn(self, which=0):
        return fsne_get_knn(self.ctx, which, self.N, self.K_hd if which == 0 else self.K_ld)

    def state(self, fields=None):
        return fsne_get_state(self.ctx, self.N, self.d, self.K_hd, self.K_ld, fields)

    def set_state(self, s):
        fsne_set_state(self.ctx, s)

    def stats(self):
        return fsne_get_stats(self.ctx)

    def sync(self):
        fsne_sync(self.ctx)

    def insert(self, Xnew, Yinit=None):
        fsne_insert_points(self.ctx, Xnew, Yinit)
        self.N += Xnew.shape[0]

    def drift(self, ids, Xnew, Yinit=None):
        fsne_drift_points(self.ctx, ids, Xnew, Yinit)

    def implode(self, factor):
        fsne_implode(self.ctx, factor)

    def delete(self, ids):
        fsne_delete_points(self.ctx, ids)
        self.N -= np.asarray(ids).size

    def renumber(self, new_of_old):
        """Point i becomes point new_of_old[i] (a permutation of 0..N-1)."""
        fsne_renumber(self.ctx, new_of_old)

    def reorder(self):
        """Renumber along the Morton curve of the embedding; returns new_of_old."""
        return fsne_reorder(self.ctx, self.N)

    def reorder_data(self):
        """Renumber along the Morton curve of a fixed projection of the data
        rows; returns new_of_old."""
        return fsne_reorder_data(self.ctx, self.N)

    def cluster(self, eps, min_pts):
        return fsne_cluster(self.ctx, self.N, eps, min_pts)

    def jump_start(self, projection=0, sigma=1e-2):
        fsne_jump_start(self.ctx, projection, sigma)

    def profile(self, enable=True):
        fsne_profile(self.ctx, enable)

    def kernel_times(self):
        return fsne_get_kernel_times(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            fsne_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


FSNE_NKERNELS = 5
KERNEL_NAMES = ("hd_refine", "affinity", "ld_grad", "reduce", "update")


def fsne_profile(ctx, enable: bool):
    L = load_library()
    L.fsne_profile.argtypes = [C.c_void_p, C.c_int32]
    L.fsne_profile.restype = C.c_int
    _check(ctx, L.fsne_profile(ctx, 1 if enable else 0))


def fsne_get_kernel_times(ctx):
    L = load_library()
    L.fsne_get_kernel_times.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.fsne_get_kernel_times.restype = C.c_int
    ms = np.zeros(FSNE_NKERNELS, dtype=np.float64)
    n = np.zeros(FSNE_NKERNELS, dtype=np.int64)
    _check(ctx, L.fsne_get_kernel_times(ctx, _ptr(ms), _ptr(n)))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_NAMES)}


# -- placement network -----------------------------------------------------------
class fsne_mlp_opts(C.Structure):
    _fields_ = [("hidden1", C.c_int32), ("hidden2", C.c_int32), ("epochs", C.c_int32),
                ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


def _mlp_lib():
    L = load_library()
    if not getattr(L, "_mlp_ready", False):
        P, I64 = C.c_void_p, C.c_int64
        L.fsne_mlp_default_opts.argtypes = [C.POINTER(fsne_mlp_opts)]
        L.fsne_mlp_create.argtypes = [P, C.POINTER(fsne_mlp_opts), C.POINTER(P)]
        L.fsne_mlp_train.argtypes = [P, P, P]
        L.fsne_mlp_predict.argtypes = [P, P, I64, P]
        L.fsne_mlp_get_params.argtypes = [P, P, P, P]
        L.fsne_mlp_set_params.argtypes = [P, P, P, P]
        L.fsne_mlp_loss_grad.argtypes = [P, P, P, I64, P, P]
        L.fsne_mlp_train_batch.argtypes = [P, P, P, I64]
        L.fsne_mlp_num_params.argtypes = [P]
        L.fsne_mlp_num_params.restype = I64
        L.fsne_mlp_destroy.argtypes = [P]
        L.fsne_mlp_destroy.restype = None
        L.fsne_mlp_last_error.argtypes = [P]
        L.fsne_mlp_last_error.restype = C.c_char_p
        for n in ("fsne_mlp_default_opts", "fsne_mlp_create", "fsne_mlp_train",
                  "fsne_mlp_predict", "fsne_mlp_get_params", "fsne_mlp_set_params",
                  "fsne_mlp_loss_grad", "fsne_mlp_train_batch"):
            getattr(L, n).restype = C.c_int
        L._mlp_ready = True
    return L


def _mcheck(m, st):
    if st != FSNE_OK:
        msg = _mlp_lib().fsne_mlp_last_error(m).decode() if m else "invalid argument"
        raise FsneError(st, msg)


def fsne_mlp_default_opts(**overrides) -> fsne_mlp_opts:
    o = fsne_mlp_opts()
    _mcheck(None, _mlp_lib().fsne_mlp_default_opts(C.byref(o)))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class Mlp:
    """Owner of one placement network (fsne_mlp_* entry points)."""

    def __init__(self, emb, opts=None):
        L = _mlp_lib()
        self.m = C.c_void_p()
        opts = opts or fsne_mlp_default_opts()
        st = L.fsne_mlp_create(emb.ctx, C.byref(opts), C.byref(self.m))
        if st != FSNE_OK:
            raise FsneError(st, "fsne_mlp_create failed")
        self.d = emb.d
        self.np = L.fsne_mlp_num_params(self.m)

    def train(self, emb):
        loss = np.zeros(1, np.float32)
        _mcheck(self.m, _mlp_lib().fsne_mlp_train(self.m, emb.ctx, _ptr(loss)))
        return float(loss[0])

    def predict(self, X):
        X = np.ascontiguousarray(X)
        Y = np.empty((X.shape[0], self.d), np.float32)
        _mcheck(self.m, _mlp_lib().fsne_mlp_predict(self.m, _ptr(X), X.shape[0], _ptr(Y)))
        return Y

    def params(self):
        p = np.empty(self.np, np.float32)
        mu = np.empty(self.d, np.float32)
        sd = np.empty(self.d, np.float32)
        _mcheck(self.m, _mlp_lib().fsne_mlp_get_params(self.m, _ptr(p), _ptr(mu), _ptr(sd)))
        return p, mu, sd

    def set_params(self, p=None, mean=None, std=None):
        a = [None if v is None else np.ascontiguousarray(v, np.float32) for v in (p, mean, std)]
        _mcheck(self.m, _mlp_lib().fsne_mlp_set_params(self.m, *[_ptr(v) for v in a]))

    def loss_grad(self, X, T):
        X = np.ascontiguousarray(X)
        T = np.ascontiguousarray(T, np.float32)
        g = np.empty(self.np, np.float32)
        loss = np.zeros(1, np.float32)
        _mcheck(self.m, _mlp_lib().fsne_mlp_loss_grad(self.m, _ptr(X), _ptr(T), X.shape[0],
                                                     _ptr(g), _ptr(loss)))
        return float(loss[0]), g

    def train_batch(self, X, T):
        X = np.ascontiguousarray(X)
        T = np.ascontiguousarray(T, np.float32)
        _mcheck(self.m, _mlp_lib().fsne_mlp_train_batch(self.m, _ptr(X), _ptr(T), X.shape[0]))

    def close(self):
        if getattr(self, "m", None):
            _mlp_lib().fsne_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
