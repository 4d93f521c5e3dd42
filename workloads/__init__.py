"""Seeded synthetic inputs (sparse matrices on lexicographic grids, right-hand
sides, serving request streams).

This package holds no arithmetic of the hierarchical method itself: it only
builds the linear systems that both the CPU oracle and the GPU library are
handed.  Every generator is deterministic given its seed.
"""

from .pde import (  # noqa: F401
    CSR,
    Problem,
    poisson2d,
    poisson3d,
    diffusion3d_expgauss,
    diffusion3d_from_coeff,
    convdiff2d_upwind,
    gaussian_field3d,
    quantized_field3d,
    vc_poisson3d,
    helmholtz3d,
    zero_diagonal_grid2d,
    rhs_uniform,
    make_config,
    config1,
    config2,
    config3,
    config4_batch,
    serving_stream,
    build_request_operator,
    Request,
    chain1d,
    random_spd_blocks,
    random_nonsym_dd,
    one_sided_dd,
    random_geometric_spd,
)
