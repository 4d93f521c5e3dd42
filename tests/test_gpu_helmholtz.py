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
