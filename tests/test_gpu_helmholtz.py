"""Indefinite systems: the paper's Helmholtz problem (Sec. 5.1, third
equation; 7-point stencil, k h = 2 pi / 32) and a more strongly indefinite
variant at 8 points per wavelength.  The pivot blocks are factored by LU
without pivoting (reading R9); on these matrices no pivot comes near zero.
Factor parity with the oracle at the bars of parity_util, and right-
preconditioned GMRES(30) to the paper's 1e-3 with the oracle's iteration
count.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from parity_util import compare_factor, solve_both
from workloads import helmholtz3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_07297_amd as P

    P.lib()
    P.config_reset()
    return P


def _relres(A, x, b):
    Asp = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    return np.linalg.norm(b - Asp @ x) / np.linalg.norm(b)


# 16^3 at 8 points per wavelength: 23 negative eigenvalues
CASES = [("exact", 0.0, 0), ("eps1e-3", 1e-3, 0), ("rank8", 1e-12, 8)]


@pytest.mark.parametrize("name,eps,K", CASES, ids=[c[0] for c in CASES])
def test_helmholtz_factor_parity(P, name, eps, K):
    A = helmholtz3d(16, 8.0)
    print(f"[helmholtz] parity {name}", flush=True)
    fo, F, st = compare_factor(P, A, (16, 16, 16), 64, eps, True, fixed_rank=K, stable_only=K > 0)
    assert st["levels_compared"] >= 2
    B, Xo, Xg = solve_both(P, torch, fo, F, A.n)
    err = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    assert err < 1e-8, err
    print(f"[helmholtz] parity {name}: {st} solve {err:.2e}", flush=True)


def test_helmholtz_gmres_matches_oracle(P):
    """24^3 at 8 points per wavelength (87 negative eigenvalues), eps 1e-3:
    GMRES(30) to 1e-3 in the oracle's number of iterations, and to 1e-10."""
    A = helmholtz3d(24, 8.0)
    b = np.random.default_rng(0).uniform(-1, 1, A.n)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, (24, 24, 24), 1e-3, 64, symmetric=1)
    fo = O.factor(A.row_ptr, A.col_idx, A.val, (24, 24, 24), 64, 1e-3, True)
    for tol in (1e-3, 1e-10):
        x, it, rel, ok = F.gmres(torch.tensor(b, device="cuda"), tol, 300, 30)
        assert ok and _relres(A, x.cpu().numpy(), b) <= tol * 1.01
        _, ito, _ = O.gmres(A.row_ptr, A.col_idx, A.val, b, lambda R: O.solve(fo, R), tol, 300)
        assert abs(it - ito) <= 1, (tol, it, ito)
        print(f"[helmholtz] 24^3 tol {tol:g}: {it} iterations (oracle {ito})", flush=True)


@pytest.mark.parametrize("side", [32, 64])
def test_helmholtz_paper_resolution(P, side):
    """32 points per wavelength (1 Hz at 32^3, 2 Hz at 64^3), fixed rank 32
    as in the paper's Helmholtz runs: GMRES(30) reaches 1e-3 within a few
    iterations, checked with an independent residual."""
    A = helmholtz3d(side)
    b = np.random.default_rng(1).uniform(-1, 1, A.n)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, (side,) * 3, 1e-12, 64, symmetric=1, fixed_rank=32)
    x, it, rel, ok = F.gmres(torch.tensor(b, device="cuda"), 1e-3, 100, 30)
    assert ok and _relres(A, x.cpu().numpy(), b) <= 1.01e-3
    assert it <= 10, it
    print(f"[helmholtz] {side}^3 K=32: {it} iterations", flush=True)


# ------------------------------------------------- partial pivoting (R16)


@pytest.mark.parametrize("nx,leaf", [(16, 8), (32, 16)])
def test_zero_diagonal_needs_pivoting(P, nx, leaf):
    """A symmetric indefinite matrix with a zero diagonal: without pivoting
    the first pivot of every block is zero (breakdown reported); with
    partial pivoting the exact mode matches the oracle's pivoted factor
    entry by entry and reproduces the dense solve."""
    from workloads import zero_diagonal_grid2d

    A = zero_diagonal_grid2d(np.random.default_rng(3), nx, nx)
    print(f"[pivoting] zero diagonal {nx}^2 leaf {leaf}", flush=True)
    with pytest.raises(P.HsError):
        P.Factor(A.row_ptr, A.col_idx, A.val, (nx, nx, 1), 0.0, leaf, symmetric=1)
    fo, F, st = compare_factor(P, A, (nx, nx, 1), leaf, 0.0, True, pivoting=1)
    B, Xo, Xg = solve_both(P, torch, fo, F, A.n)
    Xd = np.linalg.solve(A.to_dense(), B)
    assert np.linalg.norm(Xg - Xd) <= 1e-11 * np.linalg.norm(Xd)
    assert np.linalg.norm(Xg - Xo) <= 1e-10 * np.linalg.norm(Xo)
    print(f"[pivoting] zero diagonal {nx}^2: {st}", flush=True)


@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_helmholtz_pivoting_parity(P, eps):
    """Helmholtz at 8 points per wavelength with partial pivoting: the
    triangular factors stay well conditioned (cond L at most a few hundred
    against 1e5 without pivoting), so the record bars of parity_util stay
    near 1e-10; solves within 1e-8 of the oracle's."""
    A = helmholtz3d(16, 8.0)
    print(f"[pivoting] helmholtz eps={eps}", flush=True)
    fo, F, st = compare_factor(P, A, (16, 16, 16), 64, eps, True, pivoting=1)
    B, Xo, Xg = solve_both(P, torch, fo, F, A.n)
    err = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    assert err < 1e-8, err
    print(f"[pivoting] helmholtz eps={eps}: {st} solve {err:.2e}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pivoting_gmres_indefinite(P, precision):
    """GMRES(30) to 1e-10 on 24^3 Helmholtz at 8 points per wavelength with a
    pivoted eps = 1e-3 factor, both storage forms, checked with an
    independent residual."""
    A = helmholtz3d(24, 8.0)
    prec = P.HS_MIXED if precision == "mixed" else P.HS_FP64
    b = np.random.default_rng(5).uniform(-1, 1, A.n)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, (24, 24, 24), 1e-3, 64, symmetric=1, precision=prec, pivoting=1)
    x, it, rel, ok = F.gmres(torch.tensor(b, device="cuda"), 1e-10, 300, 30)
    assert ok and _relres(A, x.cpu().numpy(), b) <= 1.01e-10
    print(f"[pivoting] gmres {precision}: {it} iterations", flush=True)
