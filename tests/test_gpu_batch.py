"""Many independent systems factored in one pass (hs_factor_batch): the
clusters of every system share each level's and colour's kernel launches
(Alg. 1 on the forest of the systems' cluster trees), and CG / GMRES keep one
recurrence per system and right-hand side.

The bar: every system's factor and Krylov numbers are those of the same
system factored alone (bit for bit, since the same kernels run on the same
data in the same order; these batches hold a few dozen clusters per colour,
far below crowded_min, so batch and lone take the same kernel variants), the
batch solve agrees with the float64 oracle's solve of each system, and every
system reaches the float64 tolerance.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from workloads import config4_batch, convdiff2d_upwind, poisson2d, poisson3d, random_spd_blocks, rhs_uniform

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


def _stack(rhs):
    return torch.tensor(np.concatenate(rhs, axis=0).T.copy(), device="cuda")


def test_batch_gmres_matches_alone_bitwise(P):
    """Four nonsymmetric upwind convection-diffusion systems of different
    sizes (hence different tree depths and dense levels), mixed form with
    float32 on every level above 2000 unknowns: the batched factor's solve and
    GMRES(30) result of each system equal the lone system's bit for bit, and
    every system reaches 1e-10."""
    sides = [40, 72, 24, 57]
    systems, rhs = [], []
    rng = np.random.default_rng(11)
    for i, s in enumerate(sides):
        A = convdiff2d_upwind(s, 10.0 + 20 * i, 0.4 + i)
        systems.append((A.row_ptr, A.col_idx, A.val, (s, s, 1)))
        rhs.append(rng.uniform(-1, 1, (A.n, 2)))
    kw = dict(eps=1e-3, leaf=64, symmetric=0, precision=P.HS_MIXED, coarse_fp64_dofs=2000)
    Fb = P.Factor.batch(systems, **kw)
    assert Fb.nsys == 4 and list(np.diff(Fb.row_off)) == [s * s for s in sides]
    Bt = _stack(rhs)
    Yb = Fb.solve(Bt).cpu().numpy()
    Xb, itb, relb, okb = Fb.gmres(Bt, 1e-10, 400, 30)
    assert okb and relb.shape == (2, 4) and np.all(relb <= 1e-10)
    Xb = Xb.cpu().numpy()
    for i, (r, c, v, d) in enumerate(systems):
        F = P.Factor(r, c, v, d, **kw)
        o0, o1 = Fb.row_off[i], Fb.row_off[i + 1]
        B = torch.tensor(rhs[i].T.copy(), device="cuda")
        assert np.array_equal(F.solve(B).cpu().numpy(), Yb[:, o0:o1]), f"solve of system {i}"
        X, it, rel, ok = F.gmres(B, 1e-10, 400, 30)
        assert ok
        assert np.array_equal(X.cpu().numpy(), Xb[:, o0:o1]), f"GMRES of system {i}"
        assert np.array_equal(rel, relb[:, i])
        A = _csr(convdiff2d_upwind(sides[i], 10.0 + 20 * i, 0.4 + i))
        Xd = spla.spsolve(A.tocsc(), rhs[i])
        assert np.linalg.norm(Xb[:, o0:o1].T - Xd) / np.linalg.norm(Xd) < 1e-8


def test_batch_pcg_matches_alone_bitwise(P):
    """Symmetric positive definite systems of three shapes (3D Poisson, a 2D
    random-weight Laplacian, 2D Poisson), float64 form, PCG with 3
    right-hand sides: lanes finish at different iterations; each system's
    result equals the lone run bit for bit."""
    rng = np.random.default_rng(5)
    mats = [(poisson3d(14, 14, 14), (14, 14, 14)), (random_spd_blocks(rng, 50, 45), (50, 45, 1)),
            (poisson2d(33, 29), (33, 29, 1))]
    systems = [(A.row_ptr, A.col_idx, A.val, d) for A, d in mats]
    rhs = [rng.uniform(-1, 1, (A.n, 3)) for A, _ in mats]
    kw = dict(eps=1e-4, leaf=64, symmetric=1)
    Fb = P.Factor.batch(systems, **kw)
    Xb, itb, relb, okb = Fb.pcg(_stack(rhs), 1e-10, 200)
    assert okb and np.all(relb <= 1e-10)
    Xb = Xb.cpu().numpy()
    its = []
    for i, (r, c, v, d) in enumerate(systems):
        F = P.Factor(r, c, v, d, **kw)
        X, it, rel, ok = F.pcg(torch.tensor(rhs[i].T.copy(), device="cuda"), 1e-10, 200)
        its.append(it)
        assert ok and np.array_equal(X.cpu().numpy(), Xb[:, Fb.row_off[i]:Fb.row_off[i + 1]])
        assert np.array_equal(rel, relb[:, i])
    assert itb == max(its)


def test_batch_solve_vs_oracle(P):
    """Float64 batch of a 2D Poisson, a 2D nonsymmetric and a 1D-thin grid at
    eps 1e-6 (direct-solver regime): each system's block of the batched solve
    agrees with the oracle's solve of that system to 1e-8."""
    rng = np.random.default_rng(9)
    mats = [(poisson2d(32, 32), (32, 32, 1), 16), (convdiff2d_upwind(20, 30.0, 1.0), (20, 20, 1), 16),
            (poisson2d(64, 3), (64, 3, 1), 16)]
    systems = [(A.row_ptr, A.col_idx, A.val, d) for A, d, _ in mats]
    rhs = [rng.uniform(-1, 1, (A.n, 1)) for A, _, _ in mats]
    Fb = P.Factor.batch(systems, eps=1e-6, leaf=16, symmetric=0)
    Yb = Fb.solve(_stack(rhs)).cpu().numpy()
    for i, (A, d, leaf) in enumerate(mats):
        fo = O.factor(A.row_ptr, A.col_idx, A.val, d, leaf, 1e-6, False)
        Xo = O.solve(fo, rhs[i])
        Y = Yb[:, Fb.row_off[i]:Fb.row_off[i + 1]].T
        assert np.linalg.norm(Y - Xo) / np.linalg.norm(Xo) < 1e-8, i


def test_batch_convdiff_sample(P):
    """The batched convection-diffusion workload (sides uniform in [64, 512],
    Peclet in [1, 100], random direction) at 24 systems, mixed form with
    float64 GMRES(30): every system converges to 1e-10 (true residual
    recomputed here with a sparse product on the host)."""
    probs = config4_batch(count=24)
    systems = [(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims) for p in probs]
    Fb = P.Factor.batch(systems, eps=1e-3, leaf=64, symmetric=0, precision=P.HS_MIXED)
    Bt = _stack([p.B for p in probs])
    X, it, rel, ok = Fb.gmres(Bt, 1e-10, 300, 30)
    assert ok and np.all(rel <= 1e-10)
    X = X.cpu().numpy()[0]
    for i, p in enumerate(probs):
        x = X[Fb.row_off[i]:Fb.row_off[i + 1]]
        r = p.B[:, 0] - _csr(p.A) @ x
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(p.B[:, 0]), i


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_factor_is_deterministic(P, precision):
    """The 24-system convection-diffusion batch factored three times gives the
    same preconditioner bit for bit (hundreds of pivot workgroups per launch
    at level 0: a regression test for results that changed from run to run
    when the pivot kernel spilled registers to scratch memory)."""
    probs = config4_batch(count=24)
    systems = [(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims) for p in probs]
    prec = P.HS_MIXED if precision == "mixed" else P.HS_FP64
    B = torch.tensor(np.random.default_rng(5).uniform(-1, 1, (1, sum(p.A.n for p in probs))), device="cuda")
    ref = None
    for rep in range(3):
        Fb = P.Factor.batch(systems, eps=1e-3, leaf=64, symmetric=0, precision=prec)
        X = Fb.solve(B)
        torch.cuda.synchronize()
        if ref is None:
            ref = X.clone()
        else:
            assert torch.equal(X, ref), rep
        Fb.free()
