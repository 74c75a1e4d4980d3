"""Seeded synthetic inputs: Gaussian overlap matrices in block-sparse form.

This package builds geometry (water clusters, helical chains), evaluates the
s-type Gaussian overlap formula and cuts the result into b x b blocks.  It holds
none of the inverse-factorization arithmetic; both the CPU oracle and the GPU
path take their inputs from here.
"""
from .overlap import (  # noqa: F401
    WATER_EXPONENTS,
    BlockMatrix,
    water_cluster,
    helix_chain,
    overlap_blocks,
    overlap_dense,
    blocks_to_dense,
    dense_to_blocks,
    random_on_pattern,
    random_symmetric_on_pattern,
    config_matrix,
    CONFIGS,
)
