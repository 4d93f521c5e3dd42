"""Equivalent launch paths of the library give the same numbers bit for bit.

* The forward solve step of a colour runs as one launch whose neighbour-update
  workgroups form z_f themselves, or (when its LDS would not fit, here forced
  by many right-hand sides) as two launches; either way each column's numbers
  are those of a solve of that column alone.
* The fill-partner and neighbour updates of a colour run in one launch, or in
  two while their profiler families are timed: the factorizations agree bit
  for bit.
* The packed neighbour offsets of a colour are computed by extra workgroups of
  its Gram launch, or by a launch of their own while the Gram or pivot family
  is timed: again the factorizations agree bit for bit.
"""

import numpy as np
import pytest

from workloads import convdiff2d_upwind, poisson3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_07297_amd as P

    P.lib()
    return P


def test_forward_step_paths_agree(P):
    """With leaves of 128 unknowns and 64 right-hand sides (the most one call
    takes) the colours of the leaf level need more LDS than the one-launch
    forward step may use and take the two-launch step.  Every column equals
    its own single-column solve, which takes the one-launch step."""
    A = poisson3d(16, 16, 16)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, (16, 16, 16), 1e-4, 128, symmetric=1)
    maxm = F.info().max_cluster
    assert 2 * maxm * min(64, 8192 // maxm) * 8 + 32768 > 150 * 1024  # the two-launch step is taken
    rng = np.random.default_rng(21)
    B = torch.tensor(rng.uniform(-1, 1, (64, A.n)), device="cuda")
    X = F.solve(B)
    for c in (0, 17, 63):
        x1 = F.solve(B[c : c + 1].contiguous())
        assert torch.equal(X[c : c + 1], x1), c


def _factor_both_ways(P, A, dims, sym, families):
    """The same factorization without profiling and while `families` are
    timed (which switches the launches under test to their separate form)."""
    F1 = P.Factor(A.row_ptr, A.col_idx, A.val, dims, 1e-3, 32, symmetric=sym, precision=P.HS_MIXED)
    P.profile_reset()
    P.profile_select(families)
    P.profile_enable(True)
    try:
        F2 = P.Factor(A.row_ptr, A.col_idx, A.val, dims, 1e-3, 32, symmetric=sym, precision=P.HS_MIXED)
    finally:
        P.profile_enable(False)
        P.profile_select("")
        P.profile_reset()
    return F1, F2


@pytest.mark.parametrize("sym", [1, 0])
def test_offsets_in_gram_launch_agree(P, sym):
    """Level ranks and solves with the offsets computed inside the Gram launch
    equal those with the offsets launched on their own."""
    if sym:
        A, dims = poisson3d(12, 12, 12), (12, 12, 12)
    else:
        A, dims = convdiff2d_upwind(48, 40.0, 0.9), (48, 48, 1)
    F1, F2 = _factor_both_ways(P, A, dims, sym, "gram")
    info = F1.info()
    for l in range(info.nlevels):
        assert np.array_equal(F1.ranks(l), F2.ranks(l)), l
    b = torch.tensor(np.random.default_rng(6).uniform(-1, 1, (2, A.n)), device="cuda")
    assert torch.equal(F1.solve(b), F2.solve(b))


@pytest.mark.parametrize("sym", [1, 0])
def test_fill_and_neighbour_update_paths_agree(P, sym):
    """Factor records and level ranks with the fused update launch equal those
    with separate launches (taken while the fill / neighbour families are
    profiled)."""
    if sym:
        A, dims = poisson3d(12, 12, 12), (12, 12, 12)
    else:
        A, dims = convdiff2d_upwind(48, 40.0, 0.9), (48, 48, 1)
    F1 = P.Factor(A.row_ptr, A.col_idx, A.val, dims, 1e-3, 32, symmetric=sym, precision=P.HS_MIXED)
    P.profile_reset()
    P.profile_select("fill,nbr")
    P.profile_enable(True)
    try:
        F2 = P.Factor(A.row_ptr, A.col_idx, A.val, dims, 1e-3, 32, symmetric=sym, precision=P.HS_MIXED)
    finally:
        P.profile_enable(False)
        P.profile_select("")
        P.profile_reset()
    info = F1.info()
    for l in range(info.nlevels):
        assert np.array_equal(F1.ranks(l), F2.ranks(l)), l
    b = torch.tensor(np.random.default_rng(5).uniform(-1, 1, (2, A.n)), device="cuda")
    assert torch.equal(F1.solve(b), F2.solve(b))
