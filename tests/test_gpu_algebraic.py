"""Factorization without a grid: the cluster tree comes from recursive
bisection of the graph of A (reading R14; the hs_geometry argument with
dim = 0), on unstructured sparse matrices.  Bars as in parity_util: sizes and
ranks bit-exact, level matrices and stored operators within 1e-10 relative at
eps = 0 and tol_eps(eps) at eps > 0, solves within 1e-8 of the oracle's;
Krylov solves to 1e-10 against a sparse direct solve.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from parity_util import compare_factor, solve_both
from workloads import poisson3d, random_geometric_spd

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


CASES = [
    ("geo_spd_exact", lambda: random_geometric_spd(np.random.default_rng(1), 1500), 48, 0.0, True),
    ("geo_spd_eps1e-3", lambda: random_geometric_spd(np.random.default_rng(1), 1500), 48, 1e-3, True),
    ("geo_nonsym_exact", lambda: random_geometric_spd(np.random.default_rng(2), 900, nonsym=0.3), 30, 0.0, False),
    ("geo_nonsym_eps1e-3", lambda: random_geometric_spd(np.random.default_rng(2), 900, nonsym=0.3), 30, 1e-3, False),
    # a gridded matrix with its grid withheld: the graph bisection alone
    ("p3d_nogrid_eps1e-4", lambda: poisson3d(10, 9, 8), 32, 1e-4, True),
]


@pytest.mark.parametrize("name,mk,leaf,eps,sym", CASES, ids=[c[0] for c in CASES])
def test_ungridded_factor_parity(P, name, mk, leaf, eps, sym):
    A = mk()
    print(f"[algebraic] {name}: n={A.n} leaf={leaf} eps={eps}", flush=True)
    fo, F, st = compare_factor(P, A, None, leaf, eps, sym)
    assert st["levels_compared"] >= 2
    B, Xo, Xg = solve_both(P, torch, fo, F, A.n)
    err = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    assert err < 1e-8, err
    print(f"[algebraic] {name}: {st} solve {err:.2e}", flush=True)


def test_ungridded_pcg(P):
    """CG preconditioned by the eps = 1e-3 factor of a 20000-unknown
    unstructured SPD matrix: 1e-10 for 4 right-hand sides, the sparse direct
    solution to 1e-8, and the oracle's PCG iteration count."""
    A = random_geometric_spd(np.random.default_rng(11), 20000)
    print(f"[algebraic] pcg n={A.n}", flush=True)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, None, 1e-3, 64, symmetric=1)
    B = np.random.default_rng(5).uniform(-1, 1, (A.n, 4))
    X, it, rel, ok = F.pcg(torch.tensor(B.T.copy(), device="cuda"), 1e-10, 200)
    assert ok and np.all(rel <= 1e-10)
    Xh = X.cpu().numpy().T
    Asp = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    Xd = spla.spsolve(Asp.tocsc(), B)
    assert np.linalg.norm(Xh - Xd) / np.linalg.norm(Xd) < 1e-8
    fo = O.factor(A.row_ptr, A.col_idx, A.val, None, 64, 1e-3, True)
    _, ito, _ = O.pcg(A.row_ptr, A.col_idx, A.val, B, lambda R_: O.solve(fo, R_), 1e-10, 200)
    assert abs(ito - it) <= 1, (ito, it)
    print(f"[algebraic] pcg it={it} oracle {ito}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ungridded_gmres(P, precision):
    """Right-preconditioned GMRES(30) on the nonsymmetric unstructured matrix
    (20000 unknowns), both storage forms: 1e-10 and the sparse direct
    solution to 1e-8."""
    A = random_geometric_spd(np.random.default_rng(12), 20000, nonsym=0.3)
    prec = P.HS_MIXED if precision == "mixed" else P.HS_FP64
    print(f"[algebraic] gmres {precision} n={A.n}", flush=True)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, None, 1e-3, 64, symmetric=0, precision=prec)
    b = np.random.default_rng(6).uniform(-1, 1, A.n)
    x, it, rel, ok = F.gmres(torch.tensor(b, device="cuda"), 1e-10, 300, 30)
    assert ok and rel[0] <= 1e-10
    Asp = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    xd = spla.spsolve(Asp.tocsc(), b)
    assert np.linalg.norm(x.cpu().numpy() - xd) / np.linalg.norm(xd) < 1e-8
    print(f"[algebraic] gmres {precision} it={it}", flush=True)


def test_ungridded_batch(P):
    """A batch mixing ungridded and gridded systems factors and solves as each
    system alone does (the batch only concatenates the level sweeps)."""
    A1 = random_geometric_spd(np.random.default_rng(21), 3000)
    A2 = poisson3d(12, 12, 12)
    Fb = P.Factor.batch([(A1.row_ptr, A1.col_idx, A1.val, None),
                         (A2.row_ptr, A2.col_idx, A2.val, (12, 12, 12))], 1e-3, 48, symmetric=1)
    F1 = P.Factor(A1.row_ptr, A1.col_idx, A1.val, None, 1e-3, 48, symmetric=1)
    F2 = P.Factor(A2.row_ptr, A2.col_idx, A2.val, (12, 12, 12), 1e-3, 48, symmetric=1)
    b = np.random.default_rng(7).uniform(-1, 1, A1.n + A2.n)
    xb = Fb.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    x1 = F1.solve(torch.tensor(b[:A1.n].copy(), device="cuda")).cpu().numpy()
    x2 = F2.solve(torch.tensor(b[A1.n:].copy(), device="cuda")).cpu().numpy()
    assert np.linalg.norm(xb[:A1.n] - x1) <= 1e-12 * np.linalg.norm(x1)
    assert np.linalg.norm(xb[A1.n:] - x2) <= 1e-12 * np.linalg.norm(x2)
