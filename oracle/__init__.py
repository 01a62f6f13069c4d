"""FUnc-SNE CPU oracle -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The HIP library never imports, links or calls it.
"""
from .oracle import *  # noqa: F401,F403
