"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, library routines, invariants, brute force), never against the
oracle itself.  CPU only."""

import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from parity_util import fill_ratio_of_c1, scaled_coupling_poisson
from workloads import (
    chain1d,
    config1,
    convdiff2d_upwind,
    poisson2d,
    poisson3d,
    random_nonsym_dd,
    random_spd_blocks,
)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _fac(A, dims, leaf, eps, sym, **kw):
    return O.factor(A.row_ptr, A.col_idx, A.val, dims, leaf, eps, sym, **kw)


def _relres(A, x, b):
    return np.linalg.norm(b - A.to_dense() @ x) / np.linalg.norm(b)


# ------------------------------------------------------------- symbolic


def test_tree_and_pattern_golden():
    g = _load("tree_grid4x4_leaf4.json")
    A = poisson2d(4, 4)
    tree, levels = O.symbolic_analysis(A.row_ptr, A.col_idx, tuple(g["dims"]), g["leaf"])
    assert tree.depth == g["depth"]
    assert [d.tolist() for d in tree.leaf_dofs] == g["leaves"]
    assert levels[0].adj == g["level0_adjacency"]
    assert levels[0].color == g["colors"]
    assert levels[0].fill == g["fill_partners"]


@pytest.mark.parametrize("dims,leaf", [((32, 32, 1), 16), ((12, 10, 7), 8), ((64, 1, 1), 4), ((5, 3, 1), 2)])
def test_tree_partitions_dofs(dims, leaf):
    tree = O.build_tree(dims, leaf)
    n = dims[0] * dims[1] * dims[2]
    allids = np.concatenate(tree.leaf_dofs)
    assert np.array_equal(np.sort(allids), np.arange(n))
    assert len(tree.leaf_dofs) == 2 ** tree.depth
    assert max(d.size for d in tree.leaf_dofs) <= max(leaf, 2 * int(np.ceil(n / 2 ** tree.depth)))
    # each leaf is a box: its ids are ascending (lexicographic order)
    for d in tree.leaf_dofs:
        assert np.all(np.diff(d) > 0)


def _bfs_dist(adj, src, cap=3):
    dist = {src: 0}
    frontier = [src]
    for d in range(1, cap + 1):
        nxt = []
        for u in frontier:
            for v in adj[u]:
                if v not in dist:
                    dist[v] = d
                    nxt.append(v)
        frontier = nxt
    return dist


@pytest.mark.parametrize("maker", ["p2", "p3", "rnd"])
def test_coloring_distance2_and_fill_in_AB2(maker):
    """Sec. 2.3: fill blocks are the non-zeros of A_B^2 missing from A_B; two
    clusters more than two apart never interact, so one colour may hold only
    clusters at distance >= 3 (checked by brute-force BFS)."""
    if maker == "p2":
        A, dims, leaf = poisson2d(24, 20), (24, 20, 1), 8
    elif maker == "p3":
        A, dims, leaf = poisson3d(8, 8, 8), (8, 8, 8), 8
    else:
        A, dims, leaf = random_nonsym_dd(np.random.default_rng(5), 16, 12), (16, 12, 1), 6
    tree, levels = O.symbolic_analysis(A.row_ptr, A.col_idx, dims, leaf)
    for lev in levels:
        adj = lev.adj
        ncl = len(adj)
        for i in range(ncl):
            dist = _bfs_dist(adj, i, 2)
            for j, d in dist.items():
                if j != i and d <= 2:
                    assert lev.color[i] != lev.color[j]
        # final pattern == pattern of A_B^2 (A_B with its diagonal)
        ab = np.eye(ncl, dtype=np.int64)
        for i in range(ncl):
            ab[i, adj[i]] = 1
        ab2 = (ab @ ab) > 0
        fin = np.zeros((ncl, ncl), dtype=bool)
        for i in range(ncl):
            fin[i, lev.final_pattern[i]] = True
        assert np.array_equal(fin, ab2)
        # every fill partner is at distance exactly 2
        for s in range(ncl):
            dist = _bfs_dist(adj, s, 2)
            for t in lev.fill[s]:
                assert dist.get(t) == 2


# --------------------------------------------------------- dense kernels


def test_lu_nopiv_closed_form_pivots():
    g = _load("chain4_leaf2.json")
    A = chain1d(6).to_dense()
    L, U = O.lu_nopiv(A)
    piv = np.diag(U)
    assert np.allclose(piv, [(i + 1) / i for i in range(1, 7)], rtol=1e-15, atol=0)
    assert np.allclose(piv[:4], g["pivots"], rtol=1e-15)
    assert np.allclose(L @ U, A, rtol=0, atol=1e-15)


def test_lu_nopiv_breakdown():
    with pytest.raises(O.Breakdown):
        O.lu_nopiv(np.array([[0.0, 1.0], [1.0, 0.0]]))
    with pytest.raises(O.Breakdown):
        O.lu_nopiv(np.array([[1.0, 2.0], [np.nan, 1.0]]))


def test_householder_complement_matches_lapack_q():
    """Reading R5 uses the LAPACK larfg convention, so the complement must be
    the trailing columns of LAPACK's complete Q (geqrf + orgqr)."""
    rng = np.random.default_rng(0)
    for m, k in [(8, 3), (16, 1), (20, 19), (12, 6)]:
        X = rng.standard_normal((m, k))
        V = O.householder_complement(X)
        Q, _ = np.linalg.qr(X, mode="complete")
        assert np.allclose(V, Q[:, k:], atol=1e-13)
        assert np.abs(V.T @ X).max() < 1e-13 * np.abs(X).max() * m
        assert np.allclose(V.T @ V, np.eye(m - k), atol=1e-14)


def test_qrcp_matches_lapack_geqp3_on_generic_matrix():
    """On a matrix with well-separated column norms the pivots, |R_jj| and R
    (up to the sign of each row) are those of LAPACK geqp3
    (scipy.linalg.qr with pivoting=True)."""
    rng = np.random.default_rng(1)
    for rows, n in [(30, 12), (12, 30)]:
        M = rng.standard_normal((rows, n)) * np.logspace(0, -3, n)[rng.permutation(n)]
        k, Rk, rdiag, piv = O.qrcp_truncated(M, 0.0)
        Q, R, P = sla.qr(M, pivoting=True, mode="economic")
        assert k == min(rows, n)
        assert np.array_equal(piv[:k], P[:k])
        assert np.allclose(rdiag, np.abs(np.diag(R))[:k], rtol=1e-12)
        sgn = np.sign(np.diag(R))[:k]
        assert np.allclose(Rk, R[:k, :] * sgn[:, None], atol=1e-12)


@pytest.mark.parametrize("eps", [1e-1, 1e-3, 1e-6, 1e-10])
def test_compression_error_bound_vs_svd(eps):
    """Eq. (lra) with the row-pivoted QR of F^T: every row residual left after
    k pivots is no larger than the rejected pivot, so
    ||F - U Z||_2 <= ||R_22||_F <= sqrt(m-k) eps |R_11|, |R_11| = largest row
    norm of F; by Eckart-Young sigma_{k+1}(F) is no larger (brute-force SVD)."""
    rng = np.random.default_rng(2)
    m, n = 24, 60
    F = (rng.standard_normal((m, 10)) * np.logspace(0, -12, 10)) @ rng.standard_normal((10, n))
    F += 1e-14 * rng.standard_normal((m, n))
    k, U, Z, rdiag, piv = O.compress_fill(F, eps)
    assert np.allclose(U.T @ U, np.eye(k), atol=1e-13)
    assert np.allclose(Z, U.T @ F)
    err = np.linalg.norm(F - U @ Z, 2)
    r11 = np.linalg.norm(F, axis=1).max()
    assert abs(rdiag[0] - r11) <= 1e-14 * r11
    assert err <= np.sqrt(m - k) * eps * r11 * (1 + 1e-10) + 1e-13 * r11
    sv = np.linalg.svd(F, compute_uv=False)
    if k < sv.size:
        assert sv[k] <= err * (1 + 1e-10) + 1e-14 * r11
    assert np.all(rdiag > eps * rdiag[0])


def test_compression_ties_go_to_lowest_position_and_fixed_rank():
    F = np.zeros((6, 4))
    F[1, 0] = 3.0
    F[4, 1] = 3.0  # same norm as row 1: tie -> row 1 first
    F[5, 2] = 1.0
    k, U, Z, rdiag, piv = O.compress_fill(F, 1e-3)
    assert k == 3 and list(piv) == [1, 4, 5]
    assert np.allclose(U @ Z, F)
    k2, *_ = O.compress_fill(F, 1e-3, fixed_rank=2)
    assert k2 == 2
    k0, *_ = O.compress_fill(np.zeros((3, 5)), 1e-3)
    assert k0 == 0


# ------------------------------------------------------------ whole method


def test_dense_base_case_is_plain_lu():
    """Alg. 1 lines 2-4: a matrix no larger than a leaf is factored densely."""
    rng = np.random.default_rng(3)
    A = random_spd_blocks(rng, 4, 3)
    fac = _fac(A, (4, 3, 1), 16, 1e-6, True)
    assert len(fac.levels) == 1
    rec = fac.levels[0].records[0]
    assert rec.kind == "full"
    assert np.allclose(rec.L @ rec.Uu, A.to_dense(), atol=1e-13)
    b = rng.standard_normal(A.n)
    assert np.allclose(O.solve(fac, b), np.linalg.solve(A.to_dense(), b), rtol=1e-12)


def test_chain_schur_golden():
    g = _load("chain4_leaf2.json")
    A = chain1d(g["n"])
    fac = _fac(A, (g["n"], 1, 1), g["leaf"], 0.0, True, keep_blocks=True)
    r0 = fac.levels[0].records[0]
    assert r0.kind == "full"
    r1 = fac.levels[0].records[1]
    assert r1.kind == "full"
    S = r1.L @ r1.Uu
    assert np.allclose(S, g["schur_after_first_cluster"], rtol=1e-15)
    piv = np.concatenate([np.diag(r0.Uu), np.diag(r1.Uu)])
    assert np.allclose(piv, g["pivots"], rtol=1e-15)


EXACT_CASES = [
    ("poisson2d", lambda r: (poisson2d(16, 12), (16, 12, 1), 8, True)),
    ("poisson3d", lambda r: (poisson3d(6, 6, 5), (6, 6, 5), 8, True)),
    ("spd_random", lambda r: (random_spd_blocks(r, 14, 9), (14, 9, 1), 6, True)),
    ("spd_random3d", lambda r: (random_spd_blocks(r, 5, 6, 4), (5, 6, 4), 7, True)),
    ("nonsym", lambda r: (random_nonsym_dd(r, 13, 11), (13, 11, 1), 6, False)),
    ("convdiff", lambda r: (convdiff2d_upwind(15, 80.0, 2.0), (15, 15, 1), 8, False)),
]


@pytest.mark.parametrize("name,mk", EXACT_CASES)
def test_exact_mode_matches_dense_solve(name, mk):
    """eps = 0 makes the factorization exact (abstract: a direct solver when
    the approximations are exact): residual <= 1e-12 against scipy's LU."""
    rng = np.random.default_rng(7)
    A, dims, leaf, sym = mk(rng)
    fac = _fac(A, dims, leaf, 0.0, sym)
    B = rng.uniform(-1, 1, (A.n, 3))
    X = O.solve(fac, B)
    Xref = sla.lu_solve(sla.lu_factor(A.to_dense()), B)
    assert np.linalg.norm(X - Xref) / np.linalg.norm(Xref) < 1e-12
    for j in range(3):
        assert _relres(A, X[:, j], B[:, j]) < 1e-12


@pytest.mark.parametrize("name,mk", EXACT_CASES)
def test_exact_mode_coarse_matrix_is_schur_complement(name, mk):
    """At eps = 0 no DOF is transformed, so after every level the coarse
    matrix equals A[D,D] - A[D,E] A[E,E]^{-1} A[E,D] with E the DOFs
    eliminated so far and D the rest (block Gaussian elimination)."""
    rng = np.random.default_rng(8)
    A, dims, leaf, sym = mk(rng)
    Ad = A.to_dense()
    fac = _fac(A, dims, leaf, 0.0, sym, keep_blocks=True)
    checked = 0
    for lev in fac.levels:
        if sum(lev.m) == 0:
            break
        M, offs = O.assemble_level_dense(lev)
        D = np.concatenate([d for d in lev.dofs])
        E = np.setdiff1d(np.arange(A.n), D)
        if E.size:
            S = Ad[np.ix_(D, D)] - Ad[np.ix_(D, E)] @ np.linalg.solve(Ad[np.ix_(E, E)], Ad[np.ix_(E, D)])
        else:
            S = Ad[np.ix_(D, D)]
        assert np.abs(M - S).max() <= 1e-12 * np.abs(S).max()
        checked += 1
    assert checked >= 2


def test_first_colour_clusters_are_block_lu_steps():
    """A cluster without fill has E_s = I (Sec. 2.2): its record is the LU of
    A_ss and E_R = L^{-1} A_sn, E_L = A_ns U^{-1}."""
    p = config1()
    A = p.A
    fac = _fac(A, p.dims, p.leaf, p.eps, True, keep_blocks=True)
    lev = fac.levels[0]
    for s in lev.sym.order:
        if lev.sym.color[s] != 0:
            break
        rec = lev.records[s]
        assert rec.kind == "full" and rec.fill == []
        Ass = lev.start_blocks[(s, s)]
        Asn = np.hstack([lev.start_blocks[(s, a)] for a in rec.nbrs])
        Ans = np.vstack([lev.start_blocks[(a, s)] for a in rec.nbrs])
        assert np.allclose(rec.L @ rec.Uu, Ass, atol=1e-14)
        assert np.allclose(rec.L @ rec.ER, Asn, atol=1e-14)
        assert np.allclose(rec.EL @ rec.Uu, Ans, atol=1e-14)


@pytest.mark.parametrize("sym", [True, False])
def test_operator_invariants(sym):
    """Sec. 2.1: V^T A_ss^{-1} U = 0, V orthonormal, U orthonormal, and the
    fine block becomes the identity under G_s: L_f^{-1} F_ff U_f^{-1} = I."""
    rng = np.random.default_rng(11)
    A = random_spd_blocks(rng, 20, 16) if sym else random_nonsym_dd(rng, 20, 16)
    fac = _fac(A, (20, 16, 1), 10, 1e-3, sym)
    n_low = 0
    for lev in fac.levels:
        for rec in lev.records:
            if rec.kind != "lowrank":
                continue
            n_low += 1
            Ass = rec.L @ rec.Uu
            Ainv = np.linalg.inv(Ass)
            scale = np.linalg.norm(Ainv, 2)
            assert np.abs(rec.VL.T @ Ainv @ rec.U).max() < 1e-12 * scale
            assert np.abs(rec.U.T @ Ainv @ rec.VR).max() < 1e-12 * scale
            assert np.allclose(rec.VL.T @ rec.VL, np.eye(rec.m - rec.k), atol=1e-13)
            assert np.allclose(rec.U.T @ rec.U, np.eye(rec.k), atol=1e-13)
            Fff = rec.VL.T @ Ainv @ rec.VR
            G = np.linalg.solve(rec.Lf, Fff) @ np.linalg.inv(rec.Uf)
            assert np.allclose(G, np.eye(rec.m - rec.k), atol=1e-10)
    assert n_low > 5


def test_same_colour_order_is_bit_identical():
    """Sec. 2.3 / Sec. 3.2: clusters of one colour are more than two apart and
    touch disjoint data, so their order must not change a single bit."""
    rng = np.random.default_rng(4)
    A = random_spd_blocks(rng, 24, 18)
    B = rng.uniform(-1, 1, (A.n, 2))
    f1 = _fac(A, (24, 18, 1), 8, 1e-4, True)
    f2 = _fac(A, (24, 18, 1), 8, 1e-4, True, shuffle_within_colors=np.random.default_rng(99))
    assert any(l1.exec_order != l2.exec_order for l1, l2 in zip(f1.levels, f2.levels))
    x1 = O.solve(f1, B)
    x2 = O.solve(f2, B)
    assert np.array_equal(x1, x2)
    for l1, l2 in zip(f1.levels, f2.levels):
        assert l1.k == l2.k


def test_chain_is_exact_for_any_eps():
    """1D chain: every fill block couples one DOF on each side, so the
    compression is exact up to rounding and any eps in [1e-12, 1) gives a
    direct solver (fill property of Sec. 2.3 with rank-1 fill)."""
    A = chain1d(256)
    b = np.random.default_rng(5).uniform(-1, 1, 256)
    for eps in [1e-12, 1e-6, 1e-2, 0.5]:
        fac = _fac(A, (256, 1, 1), 4, eps, True)
        x = O.solve(fac, b)
        assert _relres(A, x, b) < 1e-12
        for lev in fac.levels:
            for rec in lev.records:
                if rec.kind == "lowrank":
                    assert rec.k <= 2


@pytest.mark.parametrize("sym", [True, False])
def test_preconditioner_symmetry_and_eps_trend(sym):
    """For a symmetric matrix the approximate factorization represents a
    symmetric matrix (A_sw and A_ws are replaced by U Z and its transpose), so
    the preconditioner is symmetric; and a smaller eps gives a more accurate
    factorization (Sec. 5.4: smaller eps, fewer iterations)."""
    rng = np.random.default_rng(6)
    A = random_spd_blocks(rng, 16, 16) if sym else random_nonsym_dd(rng, 16, 16)
    Ad = A.to_dense()
    errs = []
    for eps in [3e-1, 1e-2, 1e-4, 1e-7]:
        fac = _fac(A, (16, 16, 1), 8, eps, sym)
        Minv = O.solve(fac, np.eye(A.n))
        if sym:
            assert np.abs(Minv - Minv.T).max() < 1e-11 * np.abs(Minv).max()
        errs.append(np.linalg.norm(Minv @ Ad - np.eye(A.n), 2))
    assert errs[-1] < 1e-5
    assert all(errs[i + 1] <= errs[i] * 1.01 for i in range(len(errs) - 1))


def test_pcg_and_gmres_converge_and_match_dense():
    rng = np.random.default_rng(12)
    A = random_spd_blocks(rng, 20, 20)
    fac = _fac(A, (20, 20, 1), 10, 1e-2, True)
    B = rng.uniform(-1, 1, (A.n, 3))
    X, it, res = O.pcg(A.row_ptr, A.col_idx, A.val, B, lambda R: O.solve(fac, R), 1e-10, 100)
    assert np.all(res <= 1e-10) and it < 40
    Xref = np.linalg.solve(A.to_dense(), B)
    assert np.linalg.norm(X - Xref) / np.linalg.norm(Xref) < 1e-7
    # exact preconditioner: one iteration
    fac0 = _fac(A, (20, 20, 1), 10, 0.0, True)
    _, it0, res0 = O.pcg(A.row_ptr, A.col_idx, A.val, B, lambda R: O.solve(fac0, R), 1e-10, 10)
    assert it0 == 1 and np.all(res0 < 1e-12)
    An = random_nonsym_dd(rng, 20, 20)
    facn = _fac(An, (20, 20, 1), 10, 1e-2, False)
    b = rng.uniform(-1, 1, An.n)
    x, itg, resg = O.gmres(An.row_ptr, An.col_idx, An.val, b, lambda R: O.solve(facn, R), 1e-10, 200)
    assert resg <= 1e-10 and itg < 60
    assert np.allclose(x, np.linalg.solve(An.to_dense(), b), rtol=1e-7, atol=1e-9)
    # unpreconditioned GMRES(30) still converges to the dense solution
    x2, _, res2 = O.gmres(An.row_ptr, An.col_idx, An.val, b, lambda R: R, 1e-10, 2000)
    assert res2 <= 1e-10


def test_config1_direct_solve_accuracy():
    """Config 1 (2D Poisson 32^2, leaves of 16, eps 1e-6) used as a direct
    solver: residual of order eps, the error shrinks with eps."""
    p = config1()
    fac = _fac(p.A, p.dims, p.leaf, p.eps, True)
    x = O.solve(fac, p.B)
    r = _relres(p.A, x[:, 0], p.B[:, 0])
    assert r < 1e-6
    assert len(fac.levels) == 7


# ------------------------------------------------------------- R12 noise floor

NOISE_FLOOR_R12 = 1e-12  # the fraction of ||A_ss||_F that reading R12 states


@pytest.mark.parametrize("factor_of_floor,expect_zero", [(0.5, True), (2.0, False), (1e6, False)])
def test_noise_floor_reading_r12(factor_of_floor, expect_zero):
    """Reading R12: fill whose largest row norm is at most 1e-12 ||A_ss||_F is
    rounding noise, k = 0; fill just above it is compressed (k > 0).  The
    ratio is placed by scaling one inter-leaf coupling, using that the fill
    B(c1, c2) = -A_10 A_00^{-1} A_02 is linear in it (computed here from the
    dense Schur complement, not by the oracle)."""
    _, leaf = scaled_coupling_poisson(1.0)
    # the ratio is linear in delta up to the O(delta^2) change of B(c1, c1)
    d0 = 1e-6
    r1 = fill_ratio_of_c1(scaled_coupling_poisson(d0)[0], leaf) / d0
    delta = factor_of_floor * NOISE_FLOOR_R12 / r1
    A, _ = scaled_coupling_poisson(delta)
    ratio = fill_ratio_of_c1(A, leaf)
    assert abs(ratio / (factor_of_floor * NOISE_FLOOR_R12) - 1.0) < 1e-6
    fo = _fac(A, (4, 4, 1), 4, 1e-6, True)
    lev = fo.levels[0]
    assert lev.sym.order[:2] == [0, 1] and lev.sym.fill[1] == [2]
    k1 = lev.k[1]
    if expect_zero:
        assert k1 == 0 and lev.records[1].kind == "full"
    else:
        assert 0 < k1 < lev.m[1] and lev.records[1].kind == "lowrank"
    # either way the factorization solves the system to eps-level accuracy
    b = np.random.default_rng(0).uniform(-1, 1, A.n)
    assert _relres(A, O.solve(fo, b), b) < 1e-5


# ------------------------------------------------- R14 partition without a grid


def test_algebraic_tree_golden():
    """Reading R14 on inputs small enough to follow by hand.  Path 0-1-...-7,
    leaf 2: breadth-first from 0 (moving to 7 does not lengthen the
    structure) gives 0..7, halves {0..3} | {4..7}, then {0,1} | {2,3} and
    {4,5} | {6,7}.  4 x 4 grid (id x + 4y), leaf 4: from 0 the levels are
    0 | 1 4 | 2 5 8 | 3 6 9 12 | ...  and 15 is no farther, so the first half
    of 0 1 4 2 5 8 3 6 9 12 ... is {0,1,2,3,4,5,6,8}; inside it the search
    moves to 3 (eccentricity 5 > 3), whose order 3 2 1 6 0 5 4 8 splits
    {1,2,3,6} | {0,4,5,8}; the other half from 7 (12 is no farther) orders
    7 11 10 15 9 14 13 12 and splits {7,10,11,15} | {9,12,13,14}."""
    A = chain1d(8)
    t = O.build_tree_algebraic(A.row_ptr, A.col_idx, 2)
    assert [d.tolist() for d in t.leaf_dofs] == [[0, 1], [2, 3], [4, 5], [6, 7]]
    A = poisson2d(4, 4)
    t = O.build_tree_algebraic(A.row_ptr, A.col_idx, 4)
    assert [d.tolist() for d in t.leaf_dofs] == [[1, 2, 3, 6], [0, 4, 5, 8], [7, 10, 11, 15], [9, 12, 13, 14]]


@pytest.mark.parametrize("n,leaf,seed", [(1500, 48, 1), (777, 20, 2), (64, 64, 3), (10, 1, 4)])
def test_algebraic_tree_partitions_balanced_and_local(n, leaf, seed):
    """Every unknown in exactly one leaf, 2^D leaves, leaf sizes the floor or
    ceiling of each halving, and a far smaller edge cut between the two
    halves of the root than a random equal split has (locality)."""
    from workloads import random_geometric_spd

    A = random_geometric_spd(np.random.default_rng(seed), n)
    t = O.build_tree_algebraic(A.row_ptr, A.col_idx, leaf)
    D = 0 if n <= leaf else int(np.ceil(np.log2(n / leaf)))
    assert t.depth == D and len(t.leaf_dofs) == 2 ** D
    assert np.array_equal(np.sort(np.concatenate(t.leaf_dofs)), np.arange(n))
    sizes = {n}
    for _ in range(D):
        sizes = {h for s in sizes for h in (s // 2, s - s // 2)}
    assert {d.size for d in t.leaf_dofs} <= sizes
    if D >= 1 and n >= 200:
        rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
        left = np.zeros(n, dtype=bool)
        for d in t.leaf_dofs[: len(t.leaf_dofs) // 2]:
            left[d] = True
        cut = np.count_nonzero(left[rows] != left[A.col_idx])
        perm = np.random.default_rng(0).permutation(n)
        rnd = np.zeros(n, dtype=bool)
        rnd[perm[: n // 2]] = True
        cut_random = np.count_nonzero(rnd[rows] != rnd[A.col_idx])
        assert cut < 0.5 * cut_random, (cut, cut_random)


def test_algebraic_tree_components_and_exact_mode():
    """A graph of two components: breadth-first orders take the component of
    the lowest vertex first (the root's left half holds 50 of the first
    component's 60 vertices, the right half the rest and all of the second);
    and the exact mode on an ungridded input still
    reproduces the dense solve."""
    from workloads import random_geometric_spd

    A1 = random_geometric_spd(np.random.default_rng(5), 60)
    A2 = random_geometric_spd(np.random.default_rng(6), 40)
    n = A1.n + A2.n
    rp = np.concatenate([A1.row_ptr, A2.row_ptr[1:] + A1.nnz])
    ci = np.concatenate([A1.col_idx, A2.col_idx + A1.n]).astype(np.int32)
    va = np.concatenate([A1.val, A2.val])
    t = O.build_tree_algebraic(rp, ci, 25)
    first = set(np.concatenate(t.leaf_dofs[:2]).tolist())
    assert len(first) == 50 and first <= set(range(60))
    assert set(range(60, 100)) <= set(np.concatenate(t.leaf_dofs[2:]).tolist())
    A = type(A1)(n, rp, ci, va)
    fo = O.factor(rp, ci, va, None, 16, 0.0, True)
    b = np.random.default_rng(0).uniform(-1, 1, n)
    assert _relres(A, O.solve(fo, b), b) < 1e-12


def test_colour_count_is_the_critical_path():
    """Reading R3's greedy distance-2 colouring, processed colour by colour:
    the dependency graph of the processing order (clusters within distance
    2, earlier position first) has exactly as many levels as there are
    colours.  (A cluster of colour c has, for every c' < c, a distance-2
    neighbour of colour c' coloured before it; following colour c - 1, c - 2,
    ... gives a chain of c + 1 clusters.)  So no schedule that keeps the
    processing order of interacting clusters can take fewer steps than the
    colours."""
    from workloads import convdiff2d_upwind, poisson3d

    for A, dims in ((poisson3d(16, 16, 16), (16, 16, 16)), (convdiff2d_upwind(128, 50.0, 0.3), (128, 128, 1))):
        _, levels = O.hs_oracle.symbolic_analysis(A.row_ptr, A.col_idx, dims, 32)
        for ls in levels:
            n = len(ls.adj)
            if n == 0:
                continue
            depth = [0] * n
            for s in ls.order:
                d2 = set(ls.adj[s])
                for t in ls.adj[s]:
                    d2.update(ls.adj[t])
                d2.discard(s)
                depth[s] = 1 + max([depth[t] for t in d2 if ls.pos[t] < ls.pos[s]], default=0)
            assert max(depth) == max(ls.color) + 1


# ------------------------------------------------- R16 partial pivoting


def test_pivoted_lu_matches_lapack():
    """Reading R16's LU with partial pivoting against LAPACK getrf (through
    scipy.linalg.lu): the same permutation and factors on random matrices
    (ties within 1e-10 do not occur there), and |L_ij| <= 1."""
    rng = np.random.default_rng(4)
    for n in (1, 5, 17, 64):
        A = rng.standard_normal((n, n))
        L, U, p = O.hs_oracle.lu_partial(A)
        Ps, Ls, Us = sla.lu(A)  # A = Ps Ls Us
        assert np.array_equal(A[p], Ps.T @ A)
        assert np.allclose(L, Ls, atol=1e-13) and np.allclose(U, Us, atol=1e-12)
        assert np.abs(L).max() <= 1.0
        assert np.allclose(L @ U, A[p], atol=1e-12)


def test_pivoting_solves_zero_diagonal_exactly():
    """A symmetric indefinite matrix with a zero diagonal: LU without pivoting
    breaks down at the first pivot of the first block (reading R9); with
    partial pivoting (R16) the exact mode reproduces the dense solve."""
    from workloads import zero_diagonal_grid2d

    for nx, leaf in ((16, 8), (32, 16)):
        A = zero_diagonal_grid2d(np.random.default_rng(3), nx, nx)
        b = np.random.default_rng(1).uniform(-1, 1, A.n)
        with pytest.raises(O.hs_oracle.Breakdown):
            O.factor(A.row_ptr, A.col_idx, A.val, (nx, nx, 1), leaf, 0.0, True)
        fo = O.factor(A.row_ptr, A.col_idx, A.val, (nx, nx, 1), leaf, 0.0, True, pivoting=True)
        xd = np.linalg.solve(A.to_dense(), b)
        assert np.linalg.norm(O.solve(fo, b) - xd) <= 1e-11 * np.linalg.norm(xd)


def test_pivoting_keeps_exact_and_compressed_solves():
    """On a nonsymmetric diagonally dominant operator partial pivoting gives
    another exact factorization (the same dense solve at eps = 0) and at
    eps = 1e-3 a preconditioner that GMRES still needs few iterations with."""
    from workloads import convdiff2d_upwind

    A = convdiff2d_upwind(40, 30.0, 0.3)
    b = np.random.default_rng(2).uniform(-1, 1, A.n)
    xd = np.linalg.solve(A.to_dense(), b)
    for piv in (False, True):
        fo = O.factor(A.row_ptr, A.col_idx, A.val, (40, 40, 1), 16, 0.0, False, pivoting=piv)
        assert np.linalg.norm(O.solve(fo, b) - xd) <= 1e-12 * np.linalg.norm(xd)
        fo = O.factor(A.row_ptr, A.col_idx, A.val, (40, 40, 1), 16, 1e-3, False, pivoting=piv)
        _, it, rel = O.gmres(A.row_ptr, A.col_idx, A.val, b, lambda R: O.solve(fo, R), 1e-10, 50)
        assert rel <= 1e-10 and it <= 6
