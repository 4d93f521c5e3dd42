"""CPU tests of the C ABI: the library loads, exports every function that
include/hs.h declares, reports errors without a device, and its symbolic
analysis (tree, A_B, colours, order, fill partners, final pattern) is
bit-identical to the oracle's independent implementation."""

import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1712_07297_amd import _lib as H
from workloads import poisson2d, poisson3d, random_nonsym_dd, convdiff2d_upwind, chain1d, one_sided_dd, random_geometric_spd


def test_library_exports_every_declared_function():
    L = H.lib()
    names = H.header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
        assert name in H._SIGS, f"{name} has no binding"
    assert "gfx950" in H.version()
    assert H.strerror(H.HS_ERR_BREAKDOWN) == "zero or non-finite pivot"


def test_argument_errors_need_no_device():
    L = H.lib()
    A = H.hs_csr(0, 0, None, None, None, 0)
    g = H.hs_geometry(1, 1, 1, 1)
    o = H.hs_opts(1e-3, 0, 64, 0, 1, 0)
    F = ctypes.c_void_p()
    assert L.hs_factor(None, ctypes.byref(g), ctypes.byref(o), None, ctypes.byref(F)) == H.HS_ERR_ARG
    assert L.hs_factor(ctypes.byref(A), ctypes.byref(g), ctypes.byref(o), None, None) == H.HS_ERR_ARG
    assert L.hs_solve(None, 1, None, 1, None, 1, None) == H.HS_ERR_ARG
    # bad CSR pattern is caught by the symbolic entry point
    rp = np.array([0, 2, 3], dtype=np.int64)
    ci = np.array([1, 0, 1], dtype=np.int32)  # unsorted row 0
    with pytest.raises(H.HsError) as e:
        H.Symbolic(rp, ci, (2, 1, 1), 1)
    assert e.value.code == H.HS_ERR_PATTERN
    with pytest.raises(H.HsError) as e:
        H.Symbolic(np.array([0, 1, 2], dtype=np.int64), np.array([0, 1], dtype=np.int32), (3, 1, 1), 1)
    assert e.value.code == H.HS_ERR_GEOMETRY


CASES = [
    ("p2d_32", lambda: (poisson2d(32, 32), (32, 32, 1), 16)),
    ("one_sided", lambda: (one_sided_dd(np.random.default_rng(7), 29, 22), (29, 22, 1), 12)),
    ("p2d_ragged", lambda: (poisson2d(37, 23), (37, 23, 1), 10)),
    ("p3d_16", lambda: (poisson3d(16, 16, 16), (16, 16, 16), 64)),
    ("p3d_ragged", lambda: (poisson3d(9, 7, 5), (9, 7, 5), 8)),
    ("nonsym", lambda: (random_nonsym_dd(np.random.default_rng(3), 21, 17), (21, 17, 1), 12)),
    ("convdiff", lambda: (convdiff2d_upwind(40, 30.0, 1.0), (40, 40, 1), 64)),
    ("chain", lambda: (chain1d(100), (100, 1, 1), 3)),
    ("tiny", lambda: (poisson2d(3, 2), (3, 2, 1), 64)),
    # no grid: the graph of A is bisected (reading R14)
    ("geo_nogrid", lambda: (random_geometric_spd(np.random.default_rng(1), 1500), None, 48)),
    ("geo_nonsym_nogrid", lambda: (random_geometric_spd(np.random.default_rng(2), 900, nonsym=0.3), None, 30)),
    ("p2d_nogrid", lambda: (poisson2d(37, 23), None, 10)),
    ("one_sided_nogrid", lambda: (one_sided_dd(np.random.default_rng(7), 29, 22), None, 12)),
    ("chain_nogrid", lambda: (chain1d(100), None, 3)),
    ("two_components_nogrid", lambda: (_two_components(), None, 20)),
]


def _two_components():
    A1 = random_geometric_spd(np.random.default_rng(5), 300)
    A2 = random_geometric_spd(np.random.default_rng(6), 200)
    rp = np.concatenate([A1.row_ptr, A2.row_ptr[1:] + A1.nnz])
    ci = np.concatenate([A1.col_idx, A2.col_idx + A1.n]).astype(np.int32)
    return type(A1)(A1.n + A2.n, rp, ci, np.concatenate([A1.val, A2.val]))


@pytest.mark.parametrize("name,mk", CASES)
def test_symbolic_bit_exact_against_oracle(name, mk):
    A, dims, leaf = mk()
    tree, levels = O.symbolic_analysis(A.row_ptr, A.col_idx, dims, leaf)
    S = H.Symbolic(A.row_ptr, A.col_idx, dims, leaf)
    assert S.nlevels == tree.nlevels == len(levels)
    leaf_of, local_of = S.leaves()
    assert np.array_equal(leaf_of, tree.cluster_of_dof)
    assert np.array_equal(local_of, tree.local_of_dof)
    for lvl, ls in enumerate(levels):
        g = S.level(lvl)
        ncl = len(ls.adj)
        assert g["nclusters"] == ncl
        assert g["colors"].tolist() == ls.color
        assert g["order"].tolist() == ls.order
        assert g["ncolors"] == max(ls.color) + 1
        for s in range(ncl):
            assert g["adj"][g["adj_ptr"][s]:g["adj_ptr"][s + 1]].tolist() == ls.adj[s]
            assert g["fill"][g["fill_ptr"][s]:g["fill_ptr"][s + 1]].tolist() == ls.fill[s]
            assert g["pat"][g["pat_ptr"][s]:g["pat_ptr"][s + 1]].tolist() == ls.final_pattern[s]
