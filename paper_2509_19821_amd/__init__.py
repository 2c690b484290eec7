"""MI355X-native GMPEA (arXiv 2509.19821): one generation of the two-population
constrained multiobjective evolutionary algorithm in hand-written HIP for gfx950,
behind the C ABI declared in include/gmpea.h.

The Python module is a thin ctypes binding: every step of the generation runs
in the library's kernels. Importing fails loudly when the library is not built
(run ``python -m paper_2509_19821_amd.build`` or ``__graft_entry__.build()``).
"""
from .gmpea import (AGG_PBI, AGG_TCHE, BUF, COPY_RUNTIME, COPY_STRIDED, COPY_WIDE,  # noqa: F401
                    COPY_WIDE_NT, FAMILY_CURVE, FAMILY_SPHERE, FRONT_FEASIBLE_ND, FRONT_POP1,
                    FRONT_POP2, OP_DE, OP_SBX, DeviceBuffer, Gmpea, GmpeaError, Pool, copy,
                    copy_probe, device_count, lattice, lib, lib_path, philox, reference_set)
