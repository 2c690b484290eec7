"""GMPEA CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct FP64 implementation of what one GMPEA
generation computes (Alg. 1 loop body and Alg. 2 of arXiv 2509.19821), plus
the quality indicators of Eqs. (14)-(15). Only ``tests/``, the package smoke
check and the CPU legs of ``bench.py`` (the ``cpu_baseline`` object and the
CPU columns of ``--sweep`` and ``--many``) may import it. The product path
(the HIP library and its binding) never imports, links or calls anything here,
and this package shares no code with it; the only module both sides use is
``cmop_inputs`` (seeded problem constants, no method arithmetic).

Modules
  core        ctypes front end of gmpea_oracle.c (Philox, weights, kNN,
              evaluation, aggregation, SBX/PM, one generation, front filter)
  dense_alg2  literal N x N transcription of Alg. 2 for tiny N (pins the pull)
  metrics     IGD, HV (2-D/3-D exact and brute force), reference fronts

Parity status: every function is pinned by the CPU tests in tests/ against
closed forms, brute force, published test vectors or invariants, except the
whole multi-generation run, which is "parity unpinned" against the paper (its
benchmark suites are unavailable) and pinned only by oracle/GPU agreement.
"""
from . import core  # noqa: F401
