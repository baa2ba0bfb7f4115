"""FP64 CPU oracle of the explicit S_N step (and of the P_N step in ``oracle.pn``) -- TEST
INFRASTRUCTURE.

Only ``tests/``, ``smoke()`` in ``__graft_entry__.py`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (``paper_2205_08417_amd``) never
imports, links or calls it, and the oracle never imports the product: the two share only
the seeded input generators, which hold none of the method's arithmetic.

Every function cites the passage of KiT-RT (arXiv 2205.08417) it follows.  Functions whose
results no independent check pins are marked "parity unpinned" in their docstrings.
"""
from .oracle import *  # noqa: F401,F403
