"""The serving request loop (hs_server_*): continuous batching of solve
requests, resident factorizations reused by operator key, admission by
device memory with least-recently-used eviction.

The bar: every request's solution equals that of its operator factored and
solved alone with the same options (bit for bit: batched systems run the
same kernels in the same order and keep their own Krylov recurrences), every
request reaches 1e-10, and the counters show reuse, batching and the memory
cap at work.
"""

import time

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import convdiff2d_upwind, diffusion3d_from_coeff, gaussian_field3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_07297_amd as P

    P.lib()
    return P


def _operator(kind, side, seed):
    if kind == "diff3d":
        g = gaussian_field3d(np.random.default_rng(seed), side, side, side, 8.0, 1.5)
        return diffusion3d_from_coeff(np.exp(g)), (side, side, side), 1
    rng = np.random.default_rng(seed)
    return convdiff2d_upwind(side, float(rng.uniform(1, 100)), float(rng.uniform(0, 2 * np.pi))), (side, side, 1), 0


def _dev(A):
    d = lambda x: torch.tensor(x, device="cuda")
    return d(A.row_ptr), d(A.col_idx), d(A.val)


def _run(P, srv, ops, plan, precision):
    tickets = []
    rng = np.random.default_rng(3)
    for i, (key, nrhs) in enumerate(plan):
        A, dims, sym = ops[key]
        B = torch.tensor(rng.uniform(-1, 1, (nrhs, A.n)), device="cuda")
        t = srv.submit(key, *_dev(A), dims, B, eps=1e-3, leaf=64, symmetric=sym, precision=precision, tol=1e-10,
                       maxit=300)
        tickets.append((t, key, B))
        if i % 3 == 2:
            time.sleep(0.01)  # later requests arrive while earlier ones run
    out = []
    for t, key, B in tickets:
        X, res = srv.wait(t)
        out.append((key, B, X, res))
    return out


def _check_alone(P, ops, out, precision):
    for key, B, X, res in out:
        A, dims, sym = ops[key]
        assert res["status"] == 0 and res["relres"] <= 1e-10, res
        F = P.Factor(*_dev(A), dims, 1e-3, 64, symmetric=sym, precision=precision)
        Xa, _, rel, ok = (F.pcg if sym else F.gmres)(B, 1e-10, 300)
        assert ok
        assert torch.equal(Xa, X), (key, res)
        Ah = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
        Xh, Bh = X.cpu().numpy(), B.cpu().numpy()
        for c in range(Bh.shape[0]):
            assert np.linalg.norm(Bh[c] - Ah @ Xh[c]) <= 1.01e-10 * np.linalg.norm(Bh[c])


def test_serving_results_equal_alone(P):
    """Twelve requests on eight operators (3D lognormal diffusion, CG; 2D
    convection-diffusion, GMRES), 1-4 right-hand sides, mixed form: each
    result equals the lone solve bit for bit; reused operators are served
    from resident factorizations; several requests share batches."""
    kinds = [("diff3d", 12, 1), ("convdiff2d", 40, 2), ("diff3d", 16, 3), ("convdiff2d", 64, 4), ("diff3d", 14, 5),
             ("convdiff2d", 33, 6), ("diff3d", 10, 7), ("convdiff2d", 50, 8)]
    ops = {k: _operator(*spec) for k, spec in enumerate(kinds)}
    plan = [(0, 1), (1, 2), (2, 3), (3, 1), (4, 4), (5, 2), (0, 2), (6, 1), (7, 3), (1, 1), (3, 2), (4, 1)]
    srv = P.Server(hbm_cap_gb=64, workers=2, max_batch=8, max_new_ops=4)
    out = _run(P, srv, ops, plan, P.HS_MIXED)
    st = srv.stats()
    srv.close()
    _check_alone(P, ops, out, P.HS_MIXED)
    assert st["completed"] == len(plan) and st["failed"] == 0
    assert st["reused"] >= 1 and st["factored_ops"] <= len(ops) + 2
    assert st["batches"] < len(plan)  # some requests were batched together
    assert 0 < st["p50_latency_s"] <= st["p99_latency_s"]
    assert max(r["batch_size"] for _, _, _, r in out) > 1


def test_serving_memory_cap_evicts(P):
    """A cap that holds about three factorizations of the six operators (set
    from one operator's measured footprint): idle ones are evicted least
    recently used first, the resident bytes never exceed the cap, and the
    results still equal the lone solves."""
    kinds = [("convdiff2d", 96, 10 + i) for i in range(6)]
    ops = {k: _operator(*spec) for k, spec in enumerate(kinds)}
    A, dims, sym = ops[0]
    F = P.Factor(*_dev(A), dims, 1e-3, 64, symmetric=sym)
    F.gmres(torch.ones((1, A.n), dtype=torch.float64, device="cuda"), 1e-10, 300)
    F.trim()
    info = F.info()
    F.free()
    # one factorization in flight (peak + Krylov vectors) and about two resident
    cap = 1.05 * info.peak_device_bytes + 44.0 * A.n * 8 + 2.5 * info.device_bytes
    plan = [(k, 1) for k in range(6)] + [(0, 1), (5, 1)]
    srv = P.Server(hbm_cap_gb=cap / 1e9, workers=1, max_batch=2, max_new_ops=1)
    out = _run(P, srv, ops, plan, P.HS_FP64)
    st = srv.stats()
    srv.close()
    _check_alone(P, ops, out, P.HS_FP64)
    assert st["completed"] == len(plan)
    assert st["evictions"] > 0
    assert st["peak_held_bytes"] <= cap
