"""MI355X-native real-space NEGF transmission (HIP kernels for gfx950).

The hot path lives in libnegf.so (C ABI in include/negf.h); this package is
its thin Python binding.  Importing the package does not load the library;
the first call does, and fails loudly if the library has not been built.
"""

from .api import (  # noqa: F401
    NEGF_CORE_AUTO,
    NEGF_CORE_MULTISHIFT,
    NEGF_CORE_PER_ENERGY,
    NEGF_DIR_LR,
    NEGF_DIR_RL,
    NEGF_FP64,
    NEGF_MIXED,
    NEGF_RECOVER_OFF,
    NEGF_RECOVER_RESTART,
    NEGF_SOLVER_COCG,
    NEGF_SOLVER_QMR,
    Diagnostics,
    NegfError,
    Operator,
    negf_apply_operator,
    negf_build_operator,
    negf_current,
    negf_eigenpairs,
    negf_solve_columns,
    negf_spectral_transmission,
    negf_transmission,
    negf_transmission_batch,
    negf_transmission_grad,
    negf_set_launch_shape,
    negf_tune,
    negf_version,
    operator_from_wire,
)
