"""MI355X-native HDG element condensation / recovery (arXiv:1807.00086, section 2.4.1).

The compute path lives in libhdg.so (HIP for gfx950, C ABI in include/hdg.h); this package
only binds it (``hdg.Solver``) and builds it (``build.build()``).
"""
from .hdg import Solver, HDGError, load_library, reference_table  # noqa: F401
