"""The allocation-free solve (hs_solve_noalloc) against hs_solve, through the
C ABI: the same sweeps in the same order on buffers cut from the library's
fixed device array, so the solutions must agree bit for bit.  Two calls in a
row, the second on a smaller system with fewer right-hand sides (the array
still holds the first call's values), a call in several passes (more columns
than the array holds at once), and the size limit reported as an error."""

import numpy as np
import pytest

from workloads import poisson2d, poisson3d, random_nonsym_dd

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


def _rhs(n, nrhs, seed):
    return torch.tensor(np.random.default_rng(seed).uniform(-1, 1, (nrhs, n)), device="cuda")


def test_noalloc_equals_solve_twice_smaller_second(P):
    A1 = poisson3d(20, 18, 16)
    F1 = P.Factor(A1.row_ptr, A1.col_idx, A1.val, (20, 18, 16), 1e-4, 64, symmetric=1, precision=P.HS_MIXED)
    A2 = random_nonsym_dd(np.random.default_rng(3), 30, 22)
    F2 = P.Factor(A2.row_ptr, A2.col_idx, A2.val, (30, 22, 1), 1e-3, 16, symmetric=0)
    for F, A, nrhs, seed in ((F1, A1, 4, 1), (F2, A2, 1, 2)):
        B = _rhs(A.n, nrhs, seed)
        X = torch.full_like(B, float("nan"))
        F.solve_noalloc(B, X)
        torch.cuda.synchronize()
        ref = F.solve(B)
        assert torch.equal(X, ref), (A.n, nrhs)


def test_noalloc_in_passes_and_vector_rhs(P):
    A = poisson2d(40, 36)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, (40, 36, 1), 1e-6, 16, symmetric=1)
    B = _rhs(A.n, 7, 4)
    ref = F.solve(B)
    try:
        # room for about two columns: the seven go in four passes
        P.config_set("noalloc_scratch_max", 2.5 * 8 * 3 * 2 * A.n)
        X = torch.empty_like(B)
        F.solve_noalloc(B, X)
        assert torch.equal(X, ref)
        x1 = torch.empty(A.n, dtype=torch.float64, device="cuda")
        F.solve_noalloc(B[0], x1)
        assert torch.equal(x1, ref[0])
    finally:
        P.config_reset()


def test_noalloc_rejects_what_does_not_fit(P):
    A = poisson2d(24, 20)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, (24, 20, 1), 1e-6, 16, symmetric=1)
    B = _rhs(A.n, 2, 5)
    X = torch.zeros_like(B)
    try:
        P.config_set("noalloc_scratch_max", 8 * A.n)  # less than one column
        with pytest.raises(P.HsError) as e:
            F.solve_noalloc(B, X)
        assert e.value.code == -5 and "per right-hand side" in str(e.value)
        assert torch.count_nonzero(X).item() == 0  # nothing was launched
    finally:
        P.config_reset()
    F.solve_noalloc(B, X)
    assert torch.equal(X, F.solve(B))
