"""ctypes binding of the FP64 C oracle (test infrastructure only).

The oracle state is a dict of numpy arrays owned here; the C functions work
on pointers into them.  ``OracleState.as_gpu_state()`` gives the same state
in the library's single-precision layout, for injection into the HIP path.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_fsne.so")

__all__ = ["build_oracle", "lib", "Hyper", "OracleState", "philox4x32_10", "coin", "E_next",
           "calibrate", "exact_P", "exact_cost", "exact_grad", "knn_exact", "hd_dist2",
           "num_threads"]


def build_oracle(force: bool = True, path: str = _LIB_PATH, defines=()) -> str:
    """Compile the C oracle with gcc into oracle/liboracle_fsne.so (or into
    path, with extra -D definitions: the planted-mistake builds of the tests)."""
    if not force and os.path.exists(path):
        return path
    srcs = [os.path.join(_HERE, f) for f in ("fsne_oracle.c", "fsne_mlp_oracle.c")]
    tmp = path + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-Wall", "-shared",
           "-fPIC", *[f"-D{d}" for d in defines], "-o", tmp, *srcs, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, path)
    return path


class _State(C.Structure):
    _fields_ = [("N", C.c_int64), ("D", C.c_int32), ("d", C.c_int32), ("K_hd", C.c_int32),
                ("K_ld", C.c_int32), ("xdtype", C.c_int32), ("seed", C.c_uint64),
                ("X", C.c_void_p), ("Y", C.c_void_p), ("V", C.c_void_p),
                ("hd_idx", C.c_void_p), ("hd_d2", C.c_void_p), ("ld_idx", C.c_void_p),
                ("beta", C.c_void_p), ("m", C.c_void_p), ("r", C.c_void_p),
                ("invS", C.c_void_p), ("P", C.c_void_p), ("flags", C.c_void_p),
                ("E", C.c_void_p), ("t", C.c_void_p), ("metric", C.c_int32)]


class _Hp(C.Structure):
    _fields_ = [("alpha", C.c_double), ("perplexity", C.c_double), ("lr", C.c_double),
                ("momentum", C.c_double), ("attr", C.c_double), ("rep", C.c_double),
                ("n_neg", C.c_int32), ("hd_mode", C.c_int32), ("e_smooth", C.c_double),
                ("p_min", C.c_double)]


class _MlpDims(C.Structure):
    _fields_ = [("D", C.c_int32), ("H1", C.c_int32), ("H2", C.c_int32), ("d", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("fired", C.c_int32), ("n_new", C.c_int64), ("Z", C.c_double),
                ("E", C.c_double), ("t", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_oracle()
        _lib = _declare(C.CDLL(_LIB_PATH))
    return _lib


@contextlib.contextmanager
def using_library(path: str):
    """Route every oracle call through another build of the oracle (a
    planted-mistake build in the tests) for the duration of the block."""
    global _lib
    saved = lib()
    _lib = _declare(C.CDLL(path))
    try:
        yield _lib
    finally:
        _lib = saved


def _declare(L):
    """Argument and result types of the oracle's C functions."""
    P = C.c_void_p
    L.fsneo_philox4x32_10.argtypes = [P, P, P]
    L.fsneo_coin.argtypes = [C.c_double, C.c_uint32, C.c_uint64, C.c_int32, C.c_double]
    L.fsneo_coin.restype = C.c_int
    L.fsneo_coin_margin.argtypes = [C.c_double, C.c_uint32, C.c_uint64, C.c_double]
    L.fsneo_coin_margin.restype = C.c_double
    L.fsneo_E_next.argtypes = [C.c_double, C.c_int64, C.c_int64, C.c_double]
    L.fsneo_E_next.restype = C.c_double
    L.fsneo_calibrate.argtypes = [P, C.c_int32, C.c_double, P]
    L.fsneo_calibrate.restype = C.c_int
    L.fsneo_hd_dist2.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.c_int64]
    L.fsneo_hd_dist2.restype = C.c_double
    L.fsneo_hd_dist2_metric.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                        C.c_int64]
    L.fsneo_hd_dist2_metric.restype = C.c_double
    L.fsneo_set_metric.argtypes = [C.POINTER(_State), C.POINTER(_Hp), C.c_int32]
    L.fsneo_set_metric.restype = C.c_int
    L.fsneo_init.argtypes = [C.POINTER(_State), C.POINTER(_Hp)]
    L.fsneo_init.restype = C.c_int
    L.fsneo_step.argtypes = [C.POINTER(_State), C.POINTER(_Hp), C.POINTER(_Stats), P, P, P]
    L.fsneo_step.restype = C.c_int
    L.fsneo_hd_refine_point.argtypes = [C.POINTER(_State), C.c_int64, C.c_uint32, P, P, P]
    L.fsneo_psym_row.argtypes = [C.POINTER(_State), C.c_int64, P]
    L.fsneo_ld_refine_grad_point.argtypes = [C.POINTER(_State), C.POINTER(_Hp), C.c_int64,
                                             C.c_uint32, P, P, P, P, P, P]
    L.fsneo_hd_finish.argtypes = [C.POINTER(_State), C.POINTER(_Hp)]
    L.fsneo_hd_finish.restype = None
    L.fsneo_ld_phase.argtypes = [C.POINTER(_State), C.POINTER(_Hp), C.c_uint32, P, P, P, P,
                                 P, P]
    L.fsneo_ld_phase.restype = None
    L.fsneo_point_step.argtypes = [C.POINTER(_State), C.POINTER(_Hp), C.c_int64, C.c_int32,
                                   P, P, P, P, P, P, P, P, P]
    L.fsneo_point_step.restype = C.c_int
    L.fsneo_exact_P.argtypes = [P, C.c_int32, C.c_int64, C.c_int32, C.c_double, P, P]
    L.fsneo_exact_cost.argtypes = [P, P, C.c_int64, C.c_int32, C.c_double]
    L.fsneo_exact_cost.restype = C.c_double
    L.fsneo_exact_grad.argtypes = [P, P, C.c_int64, C.c_int32, C.c_double, P]
    L.fsneo_knn_exact.argtypes = [P, C.c_int32, C.c_int64, C.c_int32, P, C.c_int64,
                                  C.c_int32, P, P]
    L.fsneo_insert.argtypes = [C.POINTER(_State), C.POINTER(_Hp), C.c_int64, P]
    L.fsneo_insert.restype = C.c_int
    L.fsneo_drift.argtypes = [C.POINTER(_State), C.POINTER(_Hp), P, C.c_int64, P]
    L.fsneo_drift.restype = C.c_int
    L.fsneo_num_threads.restype = C.c_int
    L.fsneo_set_num_threads.argtypes = [C.c_int]
    L.fsneo_set_num_threads.restype = None
    L.fsneo_jump_start.argtypes = [C.POINTER(_State), C.c_int32, C.c_double]
    L.fsneo_jump_start.restype = C.c_int
    L.fsneo_delete_fix.argtypes = [C.POINTER(_State), C.POINTER(_Hp), P]
    L.fsneo_delete_fix.restype = None
    L.fsneo_cluster.argtypes = [C.POINTER(_State), C.c_float, C.c_int32, P]
    L.fsneo_cluster.restype = C.c_int32
    L.fsneo_mlp_nparams.argtypes = [C.POINTER(_MlpDims)]
    L.fsneo_mlp_nparams.restype = C.c_int64
    L.fsneo_mlp_init.argtypes = [C.POINTER(_MlpDims), C.c_uint64, P]
    L.fsneo_mlp_forward.argtypes = [C.POINTER(_MlpDims), P, P, C.c_int32, C.c_int64,
                                    C.c_int32, P]
    L.fsneo_mlp_loss_grad.argtypes = [C.POINTER(_MlpDims), P, P, C.c_int32, P, C.c_int64,
                                      C.c_int32, P]
    L.fsneo_mlp_loss_grad.restype = C.c_double
    L.fsneo_mlp_adam.argtypes = [C.c_int64, P, P, P, P, C.c_int64, C.c_double, C.c_double,
                                 C.c_double, C.c_double]
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return lib().fsneo_num_threads()


def set_num_threads(n: int) -> None:
    lib().fsneo_set_num_threads(int(n))


class Hyper:
    """Hyperparameters of the step (same fields as the library's)."""

    def __init__(self, alpha=1.0, perplexity=10.0, lr=100.0, momentum=0.5, attr=1.0, rep=1.0,
                 n_neg=8, hd_mode=0, e_smooth=0.1, p_min=0.05):
        self.alpha, self.perplexity, self.lr, self.momentum = alpha, perplexity, lr, momentum
        self.attr, self.rep, self.n_neg, self.hd_mode = attr, rep, n_neg, hd_mode
        self.e_smooth, self.p_min = e_smooth, p_min

    def c(self) -> _Hp:
        return _Hp(self.alpha, self.perplexity, self.lr, self.momentum, self.attr, self.rep,
                   int(self.n_neg), int(self.hd_mode), float(self.e_smooth), float(self.p_min))

    def copy(self, **kw):
        h = Hyper(**self.__dict__)
        for k, v in kw.items():
            setattr(h, k, v)
        return h


def _xprep(X):
    """X as passed to C: float32 rows, or uint16 bfloat16 bit patterns."""
    X = np.ascontiguousarray(X)
    if X.dtype == np.float32:
        return X, 0
    if X.dtype == np.uint16:
        return X, 1
    raise TypeError("X must be float32 or uint16 (bfloat16 bits)")


class OracleState:
    """The oracle's full iteration state (double precision)."""

    def __init__(self, X, d, K_hd, K_ld, seed, Y0, capacity=None, metric=0):
        self.X, self.xdtype = _xprep(X)
        N, D = self.X.shape
        cap = N if capacity is None else capacity
        if cap > N:
            Xc = np.zeros((cap, D), dtype=self.X.dtype)
            Xc[:N] = self.X
            self.X = Xc
        self.N, self.D, self.d, self.K_hd, self.K_ld, self.seed = N, D, d, K_hd, K_ld, seed
        self.cap = cap
        self.Y = np.zeros((cap, d), dtype=np.float64)
        self.Y[:N] = np.asarray(Y0, dtype=np.float64)
        self.V = np.zeros((cap, d), dtype=np.float64)
        self.hd_idx = np.zeros((cap, K_hd), dtype=np.int32)
        self.hd_d2 = np.zeros((cap, K_hd), dtype=np.float64)
        self.ld_idx = np.zeros((cap, K_ld), dtype=np.int32)
        self.beta = np.zeros(cap)
        self.m = np.zeros(cap)
        self.r = np.zeros(cap)
        self.invS = np.zeros(cap)
        self.P = np.zeros((cap, K_hd))
        self.flags = np.zeros(cap, dtype=np.uint8)
        self.E = np.ones(1, dtype=np.float64)
        self.t = np.zeros(1, dtype=np.uint32)
        self.metric = int(metric)   # HD distance: 0 squared Euclidean, 1 angular

    def cstate(self) -> _State:
        return _State(self.N, self.D, self.d, self.K_hd, self.K_ld, self.xdtype, self.seed,
                      self.X.ctypes.data, self.Y.ctypes.data, self.V.ctypes.data,
                      self.hd_idx.ctypes.data, self.hd_d2.ctypes.data, self.ld_idx.ctypes.data,
                      self.beta.ctypes.data, self.m.ctypes.data, self.r.ctypes.data,
                      self.invS.ctypes.data, self.P.ctypes.data, self.flags.ctypes.data,
                      self.E.ctypes.data, self.t.ctypes.data, self.metric)

    # -- the method ---------------------------------------------------------
    def init(self, hp: Hyper):
        s = self.cstate()
        rc = lib().fsneo_init(C.byref(s), C.byref(hp.c()))
        if rc != 0:
            raise ValueError(f"fsneo_init failed ({rc})")
        return self

    def step(self, hp: Hyper, want_partials=False):
        s = self.cstate()
        st = _Stats()
        N, d = self.N, self.d
        A = R = Zh = None
        if want_partials:
            A = np.zeros((N, d))
            R = np.zeros((N, d))
            Zh = np.zeros(N)
        rc = lib().fsneo_step(C.byref(s), C.byref(hp.c()), C.byref(st),
                              None if A is None else _p(A), None if R is None else _p(R),
                              None if Zh is None else _p(Zh))
        if rc != 0:
            raise RuntimeError(f"fsneo_step failed ({rc})")
        out = dict(fired=st.fired, n_new=st.n_new, Z=st.Z, E=st.E, t=st.t)
        if want_partials:
            out.update(A=A, R=R, Zh=Zh)
        return out

    def hd_finish(self, hp: Hyper):
        """End of the HD phase on the current lists: recalibrate the flagged
        points, then recompute P for every point."""
        s = self.cstate()
        lib().fsneo_hd_finish(C.byref(s), C.byref(hp.c()))

    def ld_phase(self, hp: Hyper, hd_next, P_next, t=None):
        """LD phase of every point (LD lists, A, R, Zh) at the current Y and LD
        lists, against the given HD lists and affinities of the iteration."""
        N, Kh, Kl, d = self.N, self.K_hd, self.K_ld, self.d
        hd_next = np.ascontiguousarray(hd_next, dtype=np.int32)
        P_next = np.ascontiguousarray(P_next, dtype=np.float64)
        assert hd_next.shape == (N, Kh) and P_next.shape == (N, Kh)
        ld = np.zeros((N, Kl), np.int32)
        A = np.zeros((N, d))
        R = np.zeros((N, d))
        Zh = np.zeros(N)
        s = self.cstate()
        lib().fsneo_ld_phase(C.byref(s), C.byref(hp.c()), int(self.t[0] if t is None else t),
                             _p(hd_next), _p(P_next), _p(ld), _p(A), _p(R), _p(Zh))
        return ld, A, R, Zh

    def round_to_f32(self):
        """Round the embedding and its velocity to single precision, so that
        the oracle and a single-precision implementation start an iteration
        from the same numbers."""
        N = self.N
        self.Y[:N] = self.Y[:N].astype(np.float32)
        self.V[:N] = self.V[:N].astype(np.float32)
        return self

    @classmethod
    def from_gpu_state(cls, X, g, d, K_hd, K_ld, seed, metric=0):
        """An oracle state holding a state read from the library (single
        precision values widened to double)."""
        N = g["Y"].shape[0]
        S = cls(X[:N], d, K_hd, K_ld, seed, g["Y"].astype(np.float64), metric=metric)
        S.V[:N] = g["V"]
        S.hd_idx[:N] = g["hd_idx"]
        S.hd_d2[:N] = g["hd_d2"]
        S.ld_idx[:N] = g["ld_idx"]
        rec = g["rec"].astype(np.float64)
        S.beta[:N], S.m[:N], S.r[:N], S.invS[:N] = rec[:, 0], rec[:, 1], rec[:, 2], rec[:, 3]
        S.P[:N] = g["P"]
        S.flags[:N] = g["flags"] & 1
        S.E[0] = g["E"]
        S.t[0] = g["t"]
        return S

    def point_step(self, hp: Hyper, i: int, fired: int):
        """Next-iteration outputs of point i alone (sampled checks at large N)."""
        K, Kl, d = self.K_hd, self.K_ld, self.d
        hi = np.zeros(K, np.int32)
        hd = np.zeros(K)
        fl = np.zeros(1, np.uint8)
        rec = np.zeros(4)
        P = np.zeros(K)
        ld = np.zeros(Kl, np.int32)
        A = np.zeros(d)
        R = np.zeros(d)
        Zh = np.zeros(1)
        s = self.cstate()
        rc = lib().fsneo_point_step(C.byref(s), C.byref(hp.c()), int(i), int(fired), _p(hi),
                                    _p(hd), _p(fl), _p(rec), _p(P), _p(ld), _p(A), _p(R), _p(Zh))
        if rc != 0:
            raise RuntimeError("fsneo_point_step failed")
        return dict(hd_idx=hi, hd_d2=hd, flag=int(fl[0]), rec=rec, P=P, ld_idx=ld, A=A, R=R,
                    Zh=float(Zh[0]))

    def hd_refine_point(self, i, t=None):
        K = self.K_hd
        hi = np.zeros(K, np.int32)
        hd = np.zeros(K)
        ch = np.zeros(1, np.uint8)
        s = self.cstate()
        lib().fsneo_hd_refine_point(C.byref(s), int(i), int(self.t[0] if t is None else t),
                                    _p(hi), _p(hd), _p(ch))
        return hi, hd, int(ch[0])

    def ld_refine_grad_point(self, hp: Hyper, i, t=None, hd_next=None, P_next=None):
        """LD phase of point i against the current HD lists and P (no HD
        phase), or against the given full HD lists and affinities."""
        Kl, d = self.K_ld, self.d
        hd_next = self.hd_idx if hd_next is None else np.ascontiguousarray(hd_next, np.int32)
        P_next = self.P if P_next is None else np.ascontiguousarray(P_next, np.float64)
        assert hd_next.shape[0] >= self.N and P_next.shape[0] >= self.N
        ld = np.zeros(Kl, np.int32)
        A = np.zeros(d)
        R = np.zeros(d)
        Zh = np.zeros(1)
        s = self.cstate()
        lib().fsneo_ld_refine_grad_point(C.byref(s), C.byref(hp.c()), int(i),
                                         int(self.t[0] if t is None else t),
                                         _p(hd_next), _p(P_next), _p(ld), _p(A), _p(R),
                                         _p(Zh))
        return ld, A, R, float(Zh[0])

    def psym_row(self, i):
        out = np.zeros(self.K_hd)
        s = self.cstate()
        lib().fsneo_psym_row(C.byref(s), int(i), _p(out))
        return out

    def insert(self, hp: Hyper, Xnew, Ynew):
        Xnew, _ = _xprep(Xnew)
        n = Xnew.shape[0]
        if self.N + n > self.cap:
            raise ValueError("capacity exceeded")
        self.X[self.N:self.N + n] = Xnew
        Yn = np.ascontiguousarray(Ynew, dtype=np.float64)
        s = self.cstate()
        lib().fsneo_insert(C.byref(s), C.byref(hp.c()), n, _p(Yn))
        self.N += n

    def drift(self, hp: Hyper, ids, Xnew, Ynew=None):
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        Xnew, _ = _xprep(Xnew)
        self.X[ids] = Xnew
        Yn = None if Ynew is None else np.ascontiguousarray(Ynew, dtype=np.float64)
        s = self.cstate()
        lib().fsneo_drift(C.byref(s), C.byref(hp.c()), _p(ids), ids.size,
                          None if Yn is None else _p(Yn))

    def set_metric(self, hp: Hyper, metric):
        """Switch the HD metric: every stored distance recomputed, rows
        re-sorted, flagged and recalibrated, P recomputed, E back to 1."""
        s = self.cstate()
        if lib().fsneo_set_metric(C.byref(s), C.byref(hp.c()), int(metric)) != 0:
            raise ValueError("metric must be 0 or 1")
        self.metric = int(metric)

    def delete(self, hp: Hyper, ids):
        """Remove points: survivors at or beyond the new N move, in increasing
        order, into the freed ids below it, in increasing order; then the
        lists are rewritten (fsneo_delete_fix)."""
        ids = np.unique(np.asarray(ids, dtype=np.int64))
        N0 = self.N
        N1 = N0 - ids.size
        dead = np.zeros(N0, bool)
        dead[ids] = True
        src = np.nonzero(~dead[N1:])[0] + N1
        dst = np.nonzero(dead[:N1])[0]
        newid = np.where(dead, -1, np.arange(N0)).astype(np.int32)
        newid[src] = dst
        for name in ("X", "Y", "V", "hd_idx", "hd_d2", "ld_idx", "beta", "m", "r", "invS",
                     "flags"):
            a = getattr(self, name)
            a[dst] = a[src]
        self.N = N1
        s = self.cstate()
        lib().fsneo_delete_fix(C.byref(s), C.byref(hp.c()), _p(newid))
        return newid

    def renumber(self, new_of_old):
        """Point i becomes point new_of_old[i]: every per-point row moves to
        its new id and every list entry is mapped (a relabelling of the state;
        nothing is recomputed)."""
        p = np.asarray(new_of_old, dtype=np.int64)
        N = self.N
        if p.shape != (N,) or not np.array_equal(np.sort(p), np.arange(N)):
            raise ValueError("not a permutation of 0..N-1")
        old_of_new = np.empty(N, dtype=np.int64)
        old_of_new[p] = np.arange(N)
        for name in ("X", "Y", "V", "hd_idx", "hd_d2", "ld_idx", "beta", "m", "r", "invS", "P",
                     "flags"):
            a = getattr(self, name)
            a[:N] = a[:N][old_of_new]
        self.hd_idx[:N] = p[self.hd_idx[:N]]
        self.ld_idx[:N] = p[self.ld_idx[:N]]

    def cluster(self, eps: float, min_pts: int):
        labels = np.empty(self.N, dtype=np.int32)
        s = self.cstate()
        nc = lib().fsneo_cluster(C.byref(s), float(eps), int(min_pts), _p(labels))
        if nc < 0:
            raise MemoryError("fsneo_cluster")
        return labels, int(nc)

    def jump_start(self, projection: int = 0, sigma: float = 1e-2):
        s = self.cstate()
        if lib().fsneo_jump_start(C.byref(s), int(projection), float(sigma)) != 0:
            raise MemoryError("fsneo_jump_start")

    # -- views --------------------------------------------------------------
    def live(self, name):
        return getattr(self, name)[: self.N]

    def as_gpu_state(self):
        """The state in the library's layout (single precision, records packed)."""
        N = self.N
        rec = np.stack([self.beta[:N], self.m[:N], self.r[:N], self.invS[:N]], axis=1)
        return dict(
            Y=self.Y[:N].astype(np.float32), V=self.V[:N].astype(np.float32),
            hd_idx=self.hd_idx[:N].copy(), hd_d2=self.hd_d2[:N].astype(np.float32),
            ld_idx=self.ld_idx[:N].copy(), rec=rec.astype(np.float32),
            P=self.P[:N].astype(np.float32), flags=self.flags[:N].copy(),
            E=float(self.E[0]), t=int(self.t[0]))

    def copy(self):
        o = OracleState.__new__(OracleState)
        for k, v in self.__dict__.items():
            o.__dict__[k] = v.copy() if isinstance(v, np.ndarray) else v
        return o


# -- free functions ----------------------------------------------------------
def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().fsneo_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def coin(E, t, seed, hd_mode=0, p_min=0.05):
    return lib().fsneo_coin(float(E), int(t), int(seed), int(hd_mode), float(p_min))


def coin_margin(E, t, seed, p_min=0.05):
    """u - p 2^32 of iteration t's draw (negative: the coin fires)."""
    return lib().fsneo_coin_margin(float(E), int(t), int(seed), float(p_min))


def E_next(E, n_new, N, lam=0.1):
    return lib().fsneo_E_next(float(E), int(n_new), int(N), float(lam))


def calibrate(d2, perplexity):
    d2 = np.ascontiguousarray(d2, dtype=np.float64)
    out = np.zeros(4)
    noroot = lib().fsneo_calibrate(_p(d2), d2.size, float(perplexity), _p(out))
    return out, bool(noroot)


def hd_dist2(X, a, b, metric=0):
    X, xdt = _xprep(X)
    if metric == 0:
        return lib().fsneo_hd_dist2(_p(X), xdt, X.shape[1], int(a), int(b))
    return lib().fsneo_hd_dist2_metric(_p(X), xdt, X.shape[1], int(metric), int(a), int(b))


def exact_P(X, perplexity):
    X, xdt = _xprep(X)
    N = X.shape[0]
    P = np.zeros((N, N))
    beta = np.zeros(N)
    lib().fsneo_exact_P(_p(X), xdt, N, X.shape[1], float(perplexity), _p(P), _p(beta))
    return P, beta


def exact_cost(P, Y, alpha):
    P = np.ascontiguousarray(P, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    return lib().fsneo_exact_cost(_p(P), _p(Y), Y.shape[0], Y.shape[1], float(alpha))


def exact_grad(P, Y, alpha):
    P = np.ascontiguousarray(P, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    G = np.zeros_like(Y)
    lib().fsneo_exact_grad(_p(P), _p(Y), Y.shape[0], Y.shape[1], float(alpha), _p(G))
    return G


def knn_exact(X, queries, K):
    X, xdt = _xprep(X)
    q = np.ascontiguousarray(queries, dtype=np.int64)
    idx = np.zeros((q.size, K), dtype=np.int32)
    d2 = np.zeros((q.size, K))
    lib().fsneo_knn_exact(_p(X), xdt, X.shape[0], X.shape[1], _p(q), q.size, int(K), _p(idx),
                          _p(d2))
    return idx, d2


# -- placement MLP ------------------------------------------------------------
class Mlp:
    """Oracle of the placement network D -> H1 -> H2 -> d (flat float32 params)."""

    def __init__(self, D, H1, H2, d, seed=0):
        self.dims = _MlpDims(D, H1, H2, d)
        self.np = lib().fsneo_mlp_nparams(C.byref(self.dims))
        self.params = np.zeros(self.np, dtype=np.float32)
        lib().fsneo_mlp_init(C.byref(self.dims), int(seed), _p(self.params))
        self.m = np.zeros(self.np)
        self.v = np.zeros(self.np)
        self.t = 0

    def forward(self, X, bf16_ops=True):
        X, xdt = _xprep(X)
        out = np.zeros((X.shape[0], self.dims.d))
        lib().fsneo_mlp_forward(C.byref(self.dims), _p(self.params), _p(X), xdt, X.shape[0],
                                int(bf16_ops), _p(out))
        return out

    def loss_grad(self, X, T, bf16_ops=True):
        X, xdt = _xprep(X)
        T = np.ascontiguousarray(T, dtype=np.float32)
        g = np.zeros(self.np)
        loss = lib().fsneo_mlp_loss_grad(C.byref(self.dims), _p(self.params), _p(X), xdt, _p(T),
                                         X.shape[0], int(bf16_ops), _p(g))
        return loss, g

    def adam(self, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        g = np.ascontiguousarray(g, dtype=np.float64)
        lib().fsneo_mlp_adam(self.np, _p(self.params), _p(self.m), _p(self.v), _p(g), self.t,
                             lr, b1, b2, eps)

    def split(self, flat=None):
        """Views W1, b1, W2, b2, W3, b3 of a flat parameter (or gradient) array."""
        f = self.params if flat is None else flat
        D, H1, H2, d = self.dims.D, self.dims.H1, self.dims.H2, self.dims.d
        sizes = [(H1, D), (H1,), (H2, H1), (H2,), (d, H2), (d,)]
        out, o = [], 0
        for s in sizes:
            n = int(np.prod(s))
            out.append(f[o:o + n].reshape(s))
            o += n
        return out
