"""Plain FP64 CPU oracle of the hierarchical low-rank elimination solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the GPU path.
"""

from .hs_oracle import (  # noqa: F401
    Breakdown,
    Tree,
    LevelSymbolic,
    build_tree,
    build_tree_algebraic,
    level0_graph,
    greedy_distance2_coloring,
    processing_order,
    simulate_level_pattern,
    symbolic_analysis,
    qrcp_truncated,
    compress_fill,
    householder_complement,
    lu_nopiv,
    factor,
    solve,
    pcg,
    gmres,
    assemble_level_dense,
    factor_flops,
)
