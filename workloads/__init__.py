"""Seeded synthetic inputs for the submatrix method (sparse SPD matrices in CSR).

This package only builds input matrices and upstream gradients. It holds none
of the method's arithmetic, so both the CPU oracle's tests and the GPU path's
tests and benchmark can draw their inputs from it.
"""
from .generators import (  # noqa: F401
    CSR,
    CONFIGS,
    make_config,
    banded_spd,
    overlap_matrix,
    mixed_density_overlap,
    diagonal_spd,
    block_diagonal_spd,
    dense_spd,
    random_sparse_spd,
    arrowhead_spd,
    upstream_gradient,
)
