"""The stream-ordered allocator hook (hs_set_allocator): the binding routes
the library's device memory through PyTorch's caching allocator; results are
bit for bit those of HIP's pool, every block goes back, on the stream it was
given for, and the hook refuses to change while a factorization exists."""

import ctypes
import gc

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
    yield P
    gc.collect()
    P.use_torch_allocator(True)


def _factor_solve(P, A, dims, sym, prec):
    F = P.Factor(A.row_ptr, A.col_idx, A.val, dims, 1e-3, 64, symmetric=sym, precision=prec)
    b = torch.tensor(np.random.default_rng(0).uniform(-1, 1, A.n), device="cuda")
    x, it, rel, ok = F.gmres(b, 1e-10, 100, 30) if not sym else F.pcg(b, 1e-10, 100)
    out = x.cpu().numpy().copy()
    F.free()
    return out, it


@pytest.mark.parametrize("case", ["p3d_fp64", "convdiff_mixed"])
def test_torch_allocator_same_results(P, case):
    if case == "p3d_fp64":
        A, dims, sym, prec = poisson3d(20, 20, 20), (20, 20, 20), 1, P.HS_FP64
    else:
        A, dims, sym, prec = convdiff2d_upwind(160, 40.0, 0.4), (160, 160, 1), 0, P.HS_MIXED
    print(f"[allocator] {case}", flush=True)
    gc.collect()
    P.use_torch_allocator(True)
    x1, it1 = _factor_solve(P, A, dims, sym, prec)
    reserved = torch.cuda.memory_reserved()
    x1b, _ = _factor_solve(P, A, dims, sym, prec)
    # the second factorization reuses the cached blocks
    assert torch.cuda.memory_reserved() <= reserved * 1.05 + (64 << 20)
    gc.collect()
    P.use_torch_allocator(False)
    x2, it2 = _factor_solve(P, A, dims, sym, prec)
    gc.collect()
    P.use_torch_allocator(True)
    assert it1 == it2
    assert np.array_equal(x1, x2) and np.array_equal(x1, x1b)


def test_every_block_returns_on_its_stream(P):
    """A counting allocator over torch's: each block is freed once, with the
    stream it was allocated for, and nothing stays out after free."""
    live, log = {}, []

    def alloc(nbytes, stream, ctx):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream or 0))
        live[p] = int(stream or 0)
        log.append(("a", int(stream or 0)))
        return p

    def free(ptr, stream, ctx):
        assert live.pop(int(ptr)) == int(stream or 0)
        torch.cuda.caching_allocator_delete(int(ptr))

    from paper_1712_07297_amd._lib import _ALLOC_FN, _FREE_FN, _check

    cbs = (_ALLOC_FN(alloc), _FREE_FN(free))
    L = P.lib()
    gc.collect()
    _check(L.hs_set_allocator(ctypes.cast(cbs[0], ctypes.c_void_p), ctypes.cast(cbs[1], ctypes.c_void_p), None), "set")
    try:
        s = torch.cuda.Stream()
        A = poisson3d(16, 16, 16)
        with torch.cuda.stream(s):
            F = P.Factor(A.row_ptr, A.col_idx, A.val, (16, 16, 16), 1e-3, 64, symmetric=1, stream=s.cuda_stream)
            b = torch.ones(A.n, dtype=torch.float64, device="cuda")
            x = F.solve(b, stream=s.cuda_stream)
        s.synchronize()
        assert log and all(st == s.cuda_stream for _, st in log)
        assert live
        # changing the allocator while a factorization exists is refused
        with pytest.raises(P.HsError):
            P.use_torch_allocator(True)
        F.free()
        assert not live, f"{len(live)} blocks not returned"
        assert torch.isfinite(x).all()
    finally:
        gc.collect()
        _check(L.hs_set_allocator(None, None, None), "reset")
        P.use_torch_allocator(True)
