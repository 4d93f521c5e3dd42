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


def tol_eps(eps, route="gram"):
    """Bar on level matrices: 1e-10 at eps = 0; at eps > 0 the weakest kept
    direction of the fill basis is resolved to about u / eps^2 on the Gram
    route and u / eps on the pivoted-QR route (Householder QR of F^T: the
    basis U = orth(P R_k^T) is as well determined as cond(P R_k^T) = |R_11| /
    |R_kk| <= 1 / eps allows), with a factor 10 for its propagation through
    the levels."""
    if eps == 0:
        return 1e-10
    return max(1e-9, 1e-13 / eps**2) if route == "gram" else max(1e-9, 1e-13 / eps)


def _perm_matrix(p, n):
    """P with (P A)[i, :] = A[p[i], :] (identity when p is None)."""
    return np.eye(n) if p is None else np.eye(n)[p]


def oracle_ops(rec):
    """T_L', T_R', E_R, E_L of an oracle record, as the library stores them
    (with pivoting, P A_ss = L U: T_L' of a block LU step is L^{-1} P)."""
    P = _perm_matrix(rec.p, rec.m)
    if rec.kind == "full":
        return np.linalg.inv(rec.L) @ P, np.linalg.inv(rec.Uu), rec.ER, rec.EL
    Ainv = np.linalg.inv(P.T @ rec.L @ rec.Uu)
    Pf = _perm_matrix(rec.pf, rec.Lf.shape[0])
    TL = np.vstack([np.linalg.solve(rec.Lf, Pf @ (rec.VL.T @ Ainv)), rec.U.T @ Ainv])
    TR = np.hstack([Ainv @ rec.VR @ np.linalg.inv(rec.Uf), Ainv @ rec.U])
    return TL, TR, rec.ER, rec.EL


def rel(a, b, scale):
    return np.abs(a - b).max() / scale if a.size else 0.0


def invariant_ops(TL, TR, ER, EL, f):
    """What a low-rank record determines independently of the basis V of the
    fine unknowns (reading R5 fixes V by LAPACK's sign convention, which
    follows rounding when a Householder pivot is near zero): the coarse rows
    U^T A_ss^{-1} of T_L' and columns A_ss^{-1} U of T_R', the fine part
    A_ss^{-1} V F_ff^{-1} V^T A_ss^{-1} = T_R'[:, :f] T_L'[:f, :] of the
    solve, and the Schur update E_L E_R of Eq. (elim)."""
    return {"TL_coarse": TL[f:, :], "TR_coarse": TR[:, f:], "fine": TR[:, :f] @ TL[:f, :], "schur": EL @ ER}


def complement_pivot_ratio(rec, sym):
    """Smallest |alpha_j| / ||x_j|| over the Householder steps of the oracle's
    complement (reading R5) of X = A_ss^{-1} U, and of A_ss^{-T} U when A is
    nonsymmetric: alpha_j is the diagonal entry of the j-th reduced column x_j.
    Near zero (a cluster whose unknowns split into parts without fill, common
    in leaves of a graph bisection) the reflector's sign, and the basis V, are
    decided by rounding."""
    H = O.hs_oracle
    sides = [H._lu_solve(rec.L, rec.Uu, rec.U, rec.p)]
    if not sym:
        sides.append(H._lu_solve_t(rec.L, rec.Uu, rec.U, rec.p))
    worst = np.inf
    for X in sides:
        R = np.array(X, dtype=np.float64)
        for j in range(R.shape[1]):
            x = R[j:, j]
            nx = np.linalg.norm(x)
            if nx > 0:
                worst = min(worst, abs(x[0]) / nx)
            v, tau, _ = H._house(x)
            R[j:, j:] -= tau * np.outer(v, v @ R[j:, j:])
    return worst


BASIS_PIVOT_MIN = 1e-10


def lu_inverse_bar(rec, level_err=0.0):
    """Bar of a record built from the inverses of the unpivoted LU factors of
    A_ss (reading R9), kappa = max(cond L, cond U): the inverse of a
    triangular matrix computed in floating point carries a relative error up
    to about m u kappa (the standard forward error bound of triangular
    inversion), and an error e in the level matrix that A_ss comes from moves
    the inverse by up to kappa e to first order; a factor 10 covers the
    operations around them.  On well-conditioned blocks this stays far below
    the 1e-10 bar; the LU of an indefinite block without pivoting can have
    cond(L) in the thousands."""
    kappa = max(np.linalg.cond(rec.L), np.linalg.cond(rec.Uu))
    return 10.0 * kappa * (rec.m * np.finfo(np.float64).eps + level_err)


def perturbed(A, rel=1e-15, seed=0):
    """A with every stored value scaled by (1 + rel r), r standard normal, the
    same r for (i, j) and (j, i): a rounding-level perturbation that keeps the
    pattern and the symmetry."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    cols = A.col_idx.astype(np.int64)
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    key = lo * A.n + hi
    uniq, inv = np.unique(key, return_inverse=True)
    r = np.random.default_rng(seed).standard_normal(uniq.size)[inv]
    return type(A)(A.n, A.row_ptr, A.col_idx, A.val * (1.0 + rel * r))


def compare_factor(P, A, dims, leaf, eps, sym, check_records=True, max_level_check=99, fixed_rank=0,
                   rec_tol=None, route=None, raw_records=None, stable_only=False, pivoting=0, **kw):
    """Factor with both; assert sizes and ranks bit-exact, level matrices and
    stored operators within the bars above.  route: "gram" or "qrcp" (the
    library's choice for these options when None: pivoted QR under a rank cap
    or below eps 1e-5 unless hs_config_set chose otherwise).

    A low-rank record whose complement has a Householder pivot below
    BASIS_PIVOT_MIN of its column (complement_pivot_ratio) is compared through
    its basis-invariant quantities only.

    stable_only: compare a level matrix or a record invariant only where the
    oracle's own value moves by less than a tenth of the bar under each of
    four rounding-level perturbations of A (perturbed()).  At small eps a pivot of the
    column-pivoted QR can be chosen between candidates whose remaining norms
    agree to within the rounding of the recomputed norms; the kept basis,
    and everything expressed in it, is then decided by rounding in both
    implementations (both choices are valid factorizations of the same
    accuracy), and only what the input determines is compared.

    Returns (oracle factor, GPU factor, statistics of what was compared)."""
    fo = O.factor(A.row_ptr, A.col_idx, A.val, dims, leaf, eps, sym, fixed_rank=fixed_rank, keep_blocks=True,
                  pivoting=bool(pivoting))
    fps = []
    if stable_only:
        for seed in range(4):
            Ap = perturbed(A, seed=seed)
            fps.append(O.factor(Ap.row_ptr, Ap.col_idx, Ap.val, dims, leaf, eps, sym, fixed_rank=fixed_rank,
                                keep_blocks=True, pivoting=bool(pivoting)))
    F = P.Factor(A.row_ptr, A.col_idx, A.val, dims, eps, leaf, symmetric=1 if sym else 0, keep_levels=True,
                 fixed_rank=fixed_rank, pivoting=pivoting, **kw)
    if route is None:
        mode = P.config_get("compression")
        route = "qrcp" if mode == 1 or (mode == 0 and (fixed_rank > 0 or eps < P.config_get("qrcp_below_eps"))) \
            else "gram"
    tol = tol_eps(eps, route)
    if rec_tol is None:
        rec_tol = tol if eps == 0 else max(tol * 100, 1e-9)
    if raw_records is None:
        raw_records = route == "gram"
    info = F.info()
    assert info.nlevels == len(fo.levels)
    stats = {"records": 0, "max_m": 0, "max_lowrank_m": 0, "max_k": 0, "worst_level": 0.0, "worst_record": 0.0,
             "worst_invariant": 0.0, "levels_compared": 0, "skipped_unstable": 0, "basis_by_rounding": 0}
    for l, lev in enumerate(fo.levels):
        assert np.array_equal(F.sizes(l), lev.m), f"sizes level {l}"
        assert np.array_equal(F.ranks(l), lev.k), f"ranks level {l}"
        stats["max_m"] = max(stats["max_m"], max(lev.m))
        if sum(lev.m) == 0 or l > max_level_check:
            continue
        Mo, _ = O.assemble_level_dense(lev)
        Mg = F.level_matrix(l)
        scale = np.abs(Mo).max()
        level_err = rel(Mg, Mo, scale)  # what the records of this level start from
        if any(not np.array_equal(fp.levels[l].m, lev.m) or
               rel(O.assemble_level_dense(fp.levels[l])[0], Mo, scale) > tol / 10 for fp in fps):
            stats["skipped_unstable"] += 1
        else:
            e = rel(Mg, Mo, scale)
            stats["worst_level"] = max(stats["worst_level"], e)
            stats["levels_compared"] += 1
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
            gops = [F.record(l, s, name) for name in ("TL", "TR", "ER", "EL")]
            base = max(1.0, np.abs(ops[0]).max())
            bar = max(rec_tol, lu_inverse_bar(rec, level_err))
            pops = []
            for fp in fps:
                rp = fp.levels[l].records[s]
                pops.append(oracle_ops(rp) if (rp.kind, rp.k) == (rec.kind, rec.k) else None)
            raw = rec.kind != "lowrank" or raw_records
            if rec.kind == "lowrank" and raw and complement_pivot_ratio(rec, sym) < BASIS_PIVOT_MIN:
                raw = False  # V decided by rounding: invariants only
                stats["basis_by_rounding"] += 1
            for q, (name, o, g) in enumerate(zip(("TL", "TR", "ER", "EL"), ops, gops)):
                assert g.shape == o.shape, (l, s, name)
                if o.size == 0 or not raw:
                    continue
                sc = max(np.abs(o).max(), 1e-8 * base)
                if any(po is None or po[q].shape != o.shape or rel(po[q], o, sc) > rec_tol / 10 for po in pops):
                    stats["skipped_unstable"] += 1
                    continue
                e = rel(g, o, sc)
                stats["worst_record"] = max(stats["worst_record"], e)
                assert e <= bar, (l, s, name, e, bar)
            if rec.kind == "lowrank":  # basis-invariant quantities, on every route
                f = rec.m - rec.k
                io, ig = invariant_ops(*ops, f), invariant_ops(*gops, f)
                ips = []
                for fp in fps:
                    rp = fp.levels[l].records[s]
                    ips.append(invariant_ops(*oracle_ops(rp), f) if (rp.kind, rp.k) == (rec.kind, rec.k) else {})
                for name in io:
                    if io[name].size == 0:
                        continue
                    sc = max(np.abs(io[name]).max(), 1e-8 * base)
                    if any(name not in ip or ip[name].shape != io[name].shape or
                           rel(ip[name], io[name], sc) > rec_tol / 10 for ip in ips):
                        stats["skipped_unstable"] += 1
                        continue
                    e = rel(ig[name], io[name], sc)
                    stats["worst_invariant"] = max(stats["worst_invariant"], e)
                    assert e <= bar, (l, s, name, e, bar)
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
