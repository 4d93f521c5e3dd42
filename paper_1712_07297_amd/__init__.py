"""Hierarchical low-rank elimination solver for sparse systems on one AMD
MI355X (gfx950): HIP kernels behind the C ABI of include/hs.h, with a thin
ctypes binding.  The factorization is the one of Chen, Pouransari,
Rajamanickam, Boman and Darve (arXiv 1712.07297), Sec. 2 (Algs. 1 and 2),
used as a direct solver or as a CG / GMRES preconditioner (Sec. 5)."""

from ._lib import (  # noqa: F401
    HS_FP64,
    HS_MIXED,
    Factor,
    HsError,
    Server,
    Symbolic,
    config_get,
    config_reset,
    config_set,
    header_functions,
    lib,
    profile_enable,
    profile_read,
    profile_reset,
    profile_select,
    strerror,
    torch_allocator_installed,
    use_torch_allocator,
    version,
)
