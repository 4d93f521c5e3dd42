"""The mixed-precision form (float32 level blocks and records, bfloat16 Schur
products accumulated in float32, float64 on the coarse levels and in every
Krylov vector) used as a preconditioner for float64 CG / GMRES (Sec. 5).

The mixed factor is not the oracle's factor (its blocks and records are
rounded to float32; its Schur products run on the bfloat16 units with every
operand split into three bfloat16 parts), so the bar is on what it is for: the
Krylov solution reaches the float64 tolerance and matches a sparse direct
solve, and the error of a single application against the float64 oracle is
measured and bounded (the bound is stated in each test).
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from workloads import config1, config2, convdiff2d_upwind

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_07297_amd as P

    P.lib()
    return P


def _csr(A):
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))


def test_mixed_pcg_poisson3d(P):
    """Config-2 shape at 16^3 with every fine level in float32: flexible PCG
    reaches 1e-10 on all 8 right-hand sides and agrees with a direct solve to
    1e-8; the stored factor is about half the float64 one."""
    p = config2(side=16, nrhs=8)
    Bt = torch.tensor(p.B.T.copy(), device="cuda")
    F64 = P.Factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.eps, p.leaf, symmetric=1)
    _, it64, _, ok64 = F64.pcg(Bt, 1e-10, 100)
    Fm = P.Factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.eps, p.leaf, symmetric=1,
                  precision=P.HS_MIXED, coarse_fp64_dofs=1)
    X, it, rel, ok = Fm.pcg(Bt, 1e-10, 100)
    assert ok64 and ok and np.all(rel <= 1e-10)
    assert it <= 3 * it64 + 5, (it, it64)
    Xh = X.cpu().numpy().T
    A = _csr(p.A)
    R = p.B - A @ Xh
    assert np.all(np.linalg.norm(R, axis=0) <= 1e-10 * np.linalg.norm(p.B, axis=0) * 1.01)
    Xd = spla.spsolve(A.tocsc(), p.B)
    assert np.linalg.norm(Xh - Xd) / np.linalg.norm(Xd) < 1e-8
    assert Fm.info().factor_bytes < 0.6 * F64.info().factor_bytes


def test_mixed_apply_error_vs_fp64_oracle(P):
    """Config 1 (2D Poisson 32x32, eps 1e-6) with float32 storage on every
    level that is not complete: one application of the mixed factor against
    the float64 oracle's solve.  Measured 6.8e-7 relative (float32 rounding
    of the stored factor); bound 1e-5.  The float64 form stays within 1e-8."""
    p = config1()
    fo = O.factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.leaf, p.eps, True)
    Xo = O.solve(fo, p.B)
    Bt = torch.tensor(p.B.T.copy(), device="cuda")
    Fm = P.Factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.eps, p.leaf, symmetric=1,
                  precision=P.HS_MIXED, coarse_fp64_dofs=1)
    Xm = Fm.solve(Bt).cpu().numpy().T
    err = np.linalg.norm(Xm - Xo) / np.linalg.norm(Xo)
    print(f"mixed-form solve vs float64 oracle: {err:.3e}")
    assert err < 1e-5
    F64 = P.Factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.eps, p.leaf, symmetric=1)
    X64 = F64.solve(Bt).cpu().numpy().T
    assert np.linalg.norm(X64 - Xo) / np.linalg.norm(Xo) < 1e-8


def test_mixed_gmres_convdiff(P):
    """Nonsymmetric upwind convection-diffusion with a mixed factor: GMRES(30)
    in float64 reaches 1e-10 and matches a direct solve to 1e-8."""
    A = convdiff2d_upwind(48, 60.0, 0.7)
    b = np.random.default_rng(3).uniform(-1, 1, A.n)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, (48, 48, 1), 1e-3, 64, symmetric=0,
                 precision=P.HS_MIXED, coarse_fp64_dofs=1)
    x, it, rel, ok = F.gmres(torch.tensor(b, device="cuda"), 1e-10, 300, 30)
    assert ok and rel[0] <= 1e-10
    xd = spla.spsolve(_csr(A).tocsc(), b)
    assert np.linalg.norm(x.cpu().numpy() - xd) / np.linalg.norm(xd) < 1e-8


def test_mixed_default_keeps_small_problems_fp64(P):
    """With the default threshold (16384 unknowns) a small problem has no
    float32 level: the mixed form gives the float64 form's solve exactly."""
    p = config1()
    Bt = torch.tensor(p.B.T.copy(), device="cuda")
    Fm = P.Factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.eps, p.leaf, symmetric=1, precision=P.HS_MIXED)
    F64 = P.Factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.eps, p.leaf, symmetric=1)
    assert np.array_equal(Fm.solve(Bt).cpu().numpy(), F64.solve(Bt).cpu().numpy())
    assert Fm.info().factor_bytes == F64.info().factor_bytes
