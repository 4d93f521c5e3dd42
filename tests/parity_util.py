"""Helpers of the GPU parity tests: run the oracle and the library on the same
input and compare everything the two must agree on.

Bars (from the method's accuracy requirements):
  * integer work (tree, colours, sizes, ranks): bit-exact;
  * factor entries at eps = 0 (every level's starting matrix and every stored
    operator): within 1e-10 relative;
  * at eps > 0 (Gram route of the rank-revealing QR): level matrices within
    tol_eps(eps) = max(1e-9, 1e-13 / eps^2) relative, stored operators within
    100 tol_eps(eps) (the Gram matrix F F^T resolves the weakest kept
    direction to about u / eps^2);
  * solves within 1e-8 relative of the oracle's.
"""

import contextlib

import numpy as np

import oracle as O


def tol_eps(eps):
    return 1e-10 if eps == 0 else max(1e-9, 1e-13 / eps**2)


def oracle_ops(rec):
    """T_L', T_R', E_R, E_L of an oracle record, as the library stores them."""
    if rec.kind == "full":
        return np.linalg.inv(rec.L), np.linalg.inv(rec.Uu), rec.ER, rec.EL
    Ainv = np.linalg.inv(rec.L @ rec.Uu)
    TL = np.vstack([np.linalg.solve(rec.Lf, rec.VL.T @ Ainv), rec.U.T @ Ainv])
    TR = np.hstack([Ainv @ rec.VR @ np.linalg.inv(rec.Uf), Ainv @ rec.U])
    return TL, TR, rec.ER, rec.EL


def rel(a, b, scale):
    return np.abs(a - b).max() / scale if a.size else 0.0


def compare_factor(P, A, dims, leaf, eps, sym, check_records=True, max_level_check=99, fixed_rank=0,
                   rec_tol=None, **kw):
    """Factor with both; assert sizes and ranks bit-exact, level matrices and
    stored operators within the bars above.  Returns (oracle factor, GPU
    factor, statistics of what was compared)."""
    fo = O.factor(A.row_ptr, A.col_idx, A.val, dims, leaf, eps, sym, fixed_rank=fixed_rank, keep_blocks=True)
    F = P.Factor(A.row_ptr, A.col_idx, A.val, dims, eps, leaf, symmetric=1 if sym else 0, keep_levels=True,
                 fixed_rank=fixed_rank, **kw)
    tol = tol_eps(eps)
    if rec_tol is None:
        rec_tol = tol if eps == 0 else max(tol * 100, 1e-9)
    info = F.info()
    assert info.nlevels == len(fo.levels)
    stats = {"records": 0, "max_m": 0, "max_lowrank_m": 0, "max_k": 0, "worst_level": 0.0, "worst_record": 0.0}
    for l, lev in enumerate(fo.levels):
        assert np.array_equal(F.sizes(l), lev.m), f"sizes level {l}"
        assert np.array_equal(F.ranks(l), lev.k), f"ranks level {l}"
        stats["max_m"] = max(stats["max_m"], max(lev.m))
        if sum(lev.m) == 0 or l > max_level_check:
            continue
        Mo, _ = O.assemble_level_dense(lev)
        Mg = F.level_matrix(l)
        scale = np.abs(Mo).max()
        e = rel(Mg, Mo, scale)
        stats["worst_level"] = max(stats["worst_level"], e)
        assert e <= tol, f"level {l} matrix differs by {e:.3e}"
        if not check_records:
            continue
        for s, rec in enumerate(lev.records):
            if rec.kind not in ("full", "lowrank"):
                continue
            if rec.kind == "lowrank":
                stats["max_lowrank_m"] = max(stats["max_lowrank_m"], rec.m)
                stats["max_k"] = max(stats["max_k"], rec.k)
            ops = oracle_ops(rec)
            base = max(1.0, np.abs(ops[0]).max())
            for name, o in zip(("TL", "TR", "ER", "EL"), ops):
                g = F.record(l, s, name)
                assert g.shape == o.shape, (l, s, name)
                if o.size == 0:
                    continue
                sc = max(np.abs(o).max(), 1e-8 * base)
                e = rel(g, o, sc)
                stats["worst_record"] = max(stats["worst_record"], e)
                assert e <= rec_tol, (l, s, name, e)
            stats["records"] += 1
    return fo, F, stats


def solve_both(P, torch, fo, F, n, nrhs=3, seed=0):
    B = np.random.default_rng(seed).uniform(-1, 1, (n, nrhs))
    Xo = O.solve(fo, B)
    Xg = F.solve(torch.tensor(B.T.copy(), device="cuda")).cpu().numpy().T
    return B, Xo, Xg


@contextlib.contextmanager
def knobs(P, **values):
    """Set kernel-variant thresholds for the duration of a block."""
    try:
        for k, v in values.items():
            P.config_set(k, v)
        yield
    finally:
        P.config_reset()


# ------------------------------------------ input of the noise-floor cases


def scaled_coupling_poisson(delta):
    """2D Poisson on a 4 x 4 grid cut into four 2 x 2 leaves (c0: x<2, y<2;
    c1: x<2, y>=2; c2: x>=2, y<2; c3: x>=2, y>=2), with every coupling between
    c0 and c1 multiplied by delta (values only; the pattern is unchanged)."""
    from workloads import poisson2d

    A = poisson2d(4, 4)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    x, y = np.arange(A.n) % 4, np.arange(A.n) // 4
    leaf = (x >= 2) * 2 + (y >= 2)
    val = A.val.copy()
    pair = {(leaf[r], leaf[c]) for r, c in zip(rows, A.col_idx)}
    assert (0, 1) in pair and (0, 3) not in pair
    sel = ((leaf[rows] == 0) & (leaf[A.col_idx] == 1)) | ((leaf[rows] == 1) & (leaf[A.col_idx] == 0))
    val[sel] *= delta
    B = type(A)(A.n, A.row_ptr, A.col_idx, val)
    return B, leaf


def fill_ratio_of_c1(A, leaf):
    """Largest row norm of the fill block B(c1, c2) that eliminating c0
    creates, over ||B(c1, c1)||_F at that time: both from the dense matrix by
    the textbook Schur complement S = A - A[:, c0] A[c0, c0]^{-1} A[c0, :]."""
    D = A.to_dense()
    i0, i1, i2 = (np.flatnonzero(leaf == c) for c in (0, 1, 2))
    S = D - D[:, i0] @ np.linalg.solve(D[np.ix_(i0, i0)], D[i0, :])
    F = S[np.ix_(i1, i2)]
    return np.linalg.norm(F, axis=1).max() / np.linalg.norm(S[np.ix_(i1, i1)])
