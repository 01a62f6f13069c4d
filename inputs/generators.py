"""Seeded synthetic workloads for the FUnc-SNE step.

This module only draws data.  It holds none of the method's arithmetic and is
shared by the CPU oracle tests, the GPU tests and the benchmark, so that both
sides of every comparison see the same bytes.

Every generator uses numpy's PCG64 with a fixed seed.  Rows are shuffled after
generation so that no structure is visible in the point index.

Workloads (shapes follow the paper's experiments, data is synthetic):

* ``blobs``       isotropic Gaussian mixture (the "Gaussian blobs" of Sec. 4.1)
* ``image_like``  sparse [0,1] images from class prototypes (MNIST-shaped, Sec. 2.3 / 4.2)
* ``manifolds``   8-dim linear manifolds in R^128 (ImageNet-scale 16/32-dim NE, Sec. 4.2)
* ``zipf_mixture`` 1000 anisotropic clusters with Zipf(1.1) sizes (heavy-tailed blobs)
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CONFIGS",
    "blobs",
    "image_like",
    "image_like_prototypes",
    "image_styles",
    "hierarchy_mixture",
    "manifolds",
    "zipf_mixture",
    "y_init",
    "f32_to_bf16_bits",
    "bf16_bits_to_f32",
    "make_workload",
]

# Per-workload method settings.  ``n_iter`` is the run length; ``alpha`` may be
# a tuple where the workload sweeps it.
CONFIGS = {
    "blobs_2k": dict(N=2000, D=50, d=2, K_hd=32, K_ld=16, n_neg=8, alpha=1.0,
                     perplexity=10.0, n_iter=500, xdtype="f32", data_seed=1001),
    "image_70k": dict(N=70000, D=784, d=2, K_hd=32, K_ld=32, n_neg=16,
                      alpha=(0.5, 1.0, 4.0), perplexity=10.0, n_iter=2000,
                      xdtype="f32", data_seed=1002),
    "manifold_1m": dict(N=1_000_000, D=128, d=16, K_hd=32, K_ld=32, n_neg=16,
                        alpha=1.0, perplexity=10.0, n_iter=1000, xdtype="bf16",
                        data_seed=1003),
    "dynamic_500k": dict(N=500_000, D=784, d=2, K_hd=32, K_ld=32, n_neg=16,
                         alpha=1.0, perplexity=10.0, n_iter=2000, xdtype="f32",
                         data_seed=1004, batches=10, batch_size=50_000,
                         drift_frac=0.01),
    "zipf_4m": dict(N=4_000_000, D=256, d=32, K_hd=64, K_ld=32, n_neg=32,
                    alpha=0.5, perplexity=20.0, n_iter=500, xdtype="bf16",
                    data_seed=1005),
}

RUN_SEED = 42


def _shuffle(rng: np.random.Generator, *arrays):
    perm = rng.permutation(arrays[0].shape[0])
    return tuple(a[perm] for a in arrays)


def blobs(n_clusters: int = 10, per_cluster: int = 200, D: int = 50,
          mean_var: float = 4.0, seed: int = 1001):
    """Isotropic Gaussian mixture: means ~ N(0, mean_var I), unit variance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.normal(0.0, np.sqrt(mean_var), size=(n_clusters, D))
    lab = np.repeat(np.arange(n_clusters), per_cluster)
    X = mu[lab] + rng.normal(0.0, 1.0, size=(lab.size, D))
    X, lab = _shuffle(rng, X.astype(np.float32), lab.astype(np.int32))
    return np.ascontiguousarray(X), lab


def image_like_prototypes(n_classes: int = 10, D: int = 784, p_on: float = 0.2,
                          seed: int = 1002):
    """Class prototypes in [0,1]^D: each pixel is on with prob p_on, value U(0.5, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    on = rng.random((n_classes, D)) < p_on
    val = rng.uniform(0.5, 1.0, size=(n_classes, D))
    return np.where(on, val, 0.0)


def image_like(n_per_class: int = 7000, n_classes: int = 10, D: int = 784,
               keep: float = 0.9, jitter: float = 0.1, seed: int = 1002,
               proto_seed: int | None = None, classes: np.ndarray | None = None):
    """Sparse image-like rows: x = clip(m * (proto + N(0, jitter^2)), 0, 1).

    ``m`` keeps each of the prototype's on-pixels with probability ``keep``;
    off-pixels stay exactly 0 (about 80% zeros overall).  ``classes`` may give
    an explicit class per row (used for insertion batches and drift).
    """
    proto = image_like_prototypes(n_classes, D, seed=seed if proto_seed is None else proto_seed)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    if classes is None:
        lab = np.repeat(np.arange(n_classes), n_per_class)
    else:
        lab = np.asarray(classes, dtype=np.int64)
    X = np.empty((lab.size, D), dtype=np.float32)
    step = 65536
    for s in range(0, lab.size, step):
        p = proto[lab[s:s + step]]
        m = (rng.random(p.shape) < keep) & (p > 0)
        x = m * (p + rng.normal(0.0, jitter, size=p.shape))
        X[s:s + step] = np.clip(x, 0.0, 1.0)
    if classes is None:
        X, lab = _shuffle(rng, X, lab.astype(np.int32))
    return np.ascontiguousarray(X), lab.astype(np.int32)


def image_styles(classes: np.ndarray, seed: int, proto_seed: int = 1002, D: int = 784,
                 k: int = 3, amp: float = 0.15, jitter: float = 0.03):
    """Image-like rows with smooth within-class variation (a "style" manifold).

    Class c has the prototype of ``image_like_prototypes`` and a style basis
    S_c (D x k, N(0, amp^2) entries on the prototype's on-pixels, 0 elsewhere);
    a row of class c is x = clip(pi_c + S_c z + N(0, jitter^2), 0, 1) on the
    on-pixels, exactly 0 off them (about 80% zeros), with z ~ N(0, I_k).
    Unlike ``image_like``, whose within-class differences are independent
    pixel drops and jitter, neighbours here follow a k-dimensional structure.
    """
    proto = image_like_prototypes(10, D, seed=proto_seed)
    on = proto > 0
    brng = np.random.Generator(np.random.PCG64(proto_seed + 31))
    S = brng.normal(0.0, amp, size=(10, D, k)) * on[:, :, None]
    lab = np.asarray(classes, dtype=np.int64)
    rng = np.random.Generator(np.random.PCG64(seed + 4973))
    z = rng.normal(size=(lab.size, k))
    X = np.empty((lab.size, D), dtype=np.float32)
    for c in range(10):
        rows = np.nonzero(lab == c)[0]
        for s0 in range(0, rows.size, 65536):
            r = rows[s0:s0 + 65536]
            x = proto[c] + z[r] @ S[c].T + rng.normal(0.0, jitter, size=(r.size, D))
            X[r] = np.where(on[c], np.clip(x, 0.0, 1.0), 0.0)
    return X, lab.astype(np.int32)


def hierarchy_mixture(n_top: int = 4, n_sub: int = 4, per_leaf: int = 1000, D: int = 50,
                      top_scale: float = 10.0, sub_scale: float = 0.6, seed: int = 1006):
    """Two-level Gaussian mixture (a hierarchy of clusters): top centres
    ~ N(0, top_scale^2 I), each with n_sub sub-centres ~ top + N(0, sub_scale^2 I),
    points ~ sub-centre + N(0, I).  Returns X (float32) and the top and leaf
    labels, rows shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed))
    top = rng.normal(0.0, top_scale, size=(n_top, D))
    sub = top[:, None, :] + rng.normal(0.0, sub_scale, size=(n_top, n_sub, D))
    leaf = np.repeat(np.arange(n_top * n_sub), per_leaf)
    X = sub.reshape(-1, D)[leaf] + rng.normal(size=(leaf.size, D))
    X, leaf = _shuffle(rng, X.astype(np.float32), leaf.astype(np.int32))
    return np.ascontiguousarray(X), (leaf // n_sub).astype(np.int32), leaf


def manifolds(n_manifolds: int = 50, per_manifold: int = 20000, D: int = 128,
              k: int = 8, noise: float = 0.05, seed: int = 1003):
    """Linear k-dim manifolds in R^D: x = c + B z + N(0, noise^2 I), B orthonormal."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.empty((n_manifolds * per_manifold, D), dtype=np.float32)
    for m in range(n_manifolds):
        B, _ = np.linalg.qr(rng.normal(size=(D, k)))
        c = rng.normal(size=D)
        z = rng.normal(size=(per_manifold, k))
        x = c + z @ B.T + rng.normal(0.0, noise, size=(per_manifold, D))
        X[m * per_manifold:(m + 1) * per_manifold] = x
    lab = np.repeat(np.arange(n_manifolds), per_manifold).astype(np.int32)
    X, lab = _shuffle(rng, X, lab)
    return np.ascontiguousarray(X), lab


def zipf_sizes(N: int, n_clusters: int, s: float):
    w = np.arange(1, n_clusters + 1, dtype=np.float64) ** (-s)
    w /= w.sum()
    sizes = np.floor(N * w).astype(np.int64)
    rem = N - int(sizes.sum())
    sizes[:rem] += 1  # the remainder goes one each to the largest clusters
    return sizes


def zipf_mixture(N: int = 4_000_000, D: int = 256, n_clusters: int = 1000,
                 s: float = 1.1, seed: int = 1005, dtype=np.float32):
    """Gaussian mixture with Zipf(s) cluster sizes and anisotropic covariances.

    Per cluster: Q = QR(Gaussian D x D), eigenvalues log-uniform in [0.01, 1],
    x = mu + Q diag(sqrt(lambda)) z, mu ~ N(0, I).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = zipf_sizes(N, n_clusters, s)
    X = np.empty((N, D), dtype=dtype)
    lab = np.empty(N, dtype=np.int32)
    o = 0
    for c in range(n_clusters):
        n = int(sizes[c])
        Q, _ = np.linalg.qr(rng.normal(size=(D, D)))
        lam = np.exp(rng.uniform(np.log(0.01), np.log(1.0), size=D))
        A = (Q * np.sqrt(lam)).astype(np.float32)
        mu = rng.normal(size=D).astype(np.float32)
        z = rng.standard_normal(size=(n, D), dtype=np.float32)
        X[o:o + n] = mu + z @ A.T
        lab[o:o + n] = c
        o += n
    perm = rng.permutation(N)
    return X[perm], lab[perm]


def y_init(N: int, d: int, var: float = 1e-4, seed: int = RUN_SEED):
    """Initial LD coordinates Y0 ~ N(0, var I), float32, row-major N x d."""
    rng = np.random.Generator(np.random.PCG64(seed + 17))
    return np.ascontiguousarray(rng.normal(0.0, np.sqrt(var), size=(N, d)).astype(np.float32))


def f32_to_bf16_bits(X: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round to nearest, ties to even); returns uint16 bits."""
    u = np.ascontiguousarray(X, dtype=np.float32).view(np.uint32)
    lsb = (u >> 16) & 1
    r = (u + np.uint32(0x7FFF) + lsb) >> 16
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = np.where(nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def bf16_bits_to_f32(B: np.ndarray) -> np.ndarray:
    return (np.asarray(B, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def make_workload(name: str, N: int | None = None):
    """Return (X float32, labels, cfg) for a named workload, optionally truncated to N rows.

    Truncation keeps the first N shuffled rows, so a small case is a uniform
    subsample of the full one.
    """
    cfg = dict(CONFIGS[name])
    seed = cfg["data_seed"]
    if name == "blobs_2k":
        X, lab = blobs(seed=seed)
    elif name == "image_70k":
        n_per = 7000 if N is None else -(-N // 10)
        X, lab = image_like(n_per_class=n_per, seed=seed)
    elif name == "dynamic_500k":
        n_per = 50000 if N is None else -(-N // 10)
        X, lab = image_like(n_per_class=n_per, seed=seed, proto_seed=CONFIGS["image_70k"]["data_seed"])
    elif name == "manifold_1m":
        per = 20000 if N is None else -(-N // 50)
        X, lab = manifolds(per_manifold=per, seed=seed)
    elif name == "zipf_4m":
        X, lab = zipf_mixture(N=cfg["N"] if N is None else N, seed=seed)
    else:
        raise KeyError(name)
    if N is not None:
        X, lab = X[:N], lab[:N]
    cfg["N"] = X.shape[0]
    return np.ascontiguousarray(X), lab, cfg
