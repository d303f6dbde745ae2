"""MI355X-native stochastic-Galerkin space-time slab operator, Vanka/GMG preconditioner and FGMRES.

The numerical work is in libsgheat.so (hand-written gfx950 HIP kernels behind the C ABI in
include/sgheat.h); this package only binds it.  Import fails if the library is not built.
"""
from .sgheat import (SG_FP64, SG_MIXED, Problem, SgError, Spec, problem_from_workload,  # noqa: F401
                     quadrature_points, LIB_PATH, EXPORTS)
