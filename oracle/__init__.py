"""FP64 CPU oracle of the submatrix method -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg import
this package. The GPU library never does.
"""
from .submat_oracle import (  # noqa: F401
    PatternError,
    validate,
    submatrix_rows,
    gather_submatrix,
    symmetrise,
    inv_root,
    root,
    eig,
    FUNCTIONS,
    check_function,
    spectral_function,
    column_of_function,
    column_of_inverse_root,
    forward,
    forward_columns,
    divided_differences,
    adjoint_column,
    adjoint,
    residual_norm,
)
