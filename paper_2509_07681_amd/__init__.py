"""FUnc-SNE per-iteration step for MI355X (gfx950): HIP kernels behind a C ABI.

``fsne`` is the ctypes binding of ``libfsne.so`` (built by ``build.py``).
"""
from . import fsne  # noqa: F401
