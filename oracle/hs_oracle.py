"""FP64 CPU oracle of the hierarchical solver of Chen, Pouransari, Rajamanickam,
Boman and Darve, "A distributed-memory hierarchical solver for general sparse
linear systems" (arXiv 1712.07297).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product library.  Plain numpy in
float64, written for readability, not speed.

What is computed (paper Sec. 2):

* a clustering of the unknowns (Sec. 2, opening; Alg. 1 "Partition the graph")
  and the block sparsity pattern A_B of Eq. (quotient);
* for every cluster s, in a colour-major order in which clusters of one colour
  are more than two apart in A_B (Sec. 2.3, Sec. 3.4), the low-rank
  elimination W_s = P_s G_s E_s of Sec. 2.1:
    - the fill blocks A_sw are compressed, A_sw = U Z + O(eps) (Eq. lra);
    - V spans the complement with V^T A_ss^{-1} U = 0;
    - the sparsification operator E_s of Eq. (scaling) decouples the fine
      DOFs V from the coarse DOFs U and from w;
    - the elimination operator G_s of Eq. (elim) eliminates the fine DOFs and
      updates the neighbour block A_nn by a Schur complement;
    - the permutation P_s of Eq. (perm) moves the coarse DOFs last;
* Alg. 1: after all clusters of a level, the coarse DOFs form the next level's
  clusters and the procedure recurses until one cluster is left, which is
  factored densely;
* Alg. 2: forward substitution with every W_i, coarse solve, backward
  substitution with every W_i^T;
* the factorization as a preconditioner in CG / GMRES (Sec. 5).

Readings of points the paper leaves open (each one is listed in the design doc):

R1  clusters: complete geometric bisection of the grid box, fixed depth
    D = ceil(log2(N / leaf)); split the longest extent (ties x, y, z), lower
    half gets floor(extent/2) planes; level l clusters are the depth D-l boxes
    numbered left to right; next-level cluster = parent box, its DOFs are the
    left child's coarse DOFs followed by the right child's.
R2  neighbours: structural pattern of the level's starting matrix,
    symmetrised; "well-separated" w = clusters that became coupled to s by
    fill during the level (Sec. 2.1: w blocks are fill-in blocks); clusters
    already processed take part through their coarse DOFs.
R3  order: greedy distance-2 colouring by ascending cluster index; clusters
    processed by (colour, index).
R4  compression: truncated Householder QR with column pivoting of F^T, i.e.
    pivoting over the unknowns of s, where F = [A_s,w1 ... A_s,wp]
    (followed by [A_w1,s^T ... A_wp,s^T] for a nonsymmetric matrix); pivot =
    largest recomputed remaining norm, ties within a relative 1e-10 of the
    squared maximum go to the lowest position in the current (exchanged)
    order; stop at the first |R_jj| <= eps |R_11|; rows of R signed so that
    R_jj > 0; U = orthonormal factor (positive diagonal) of P R_k^T, the
    first k columns of R^T put back in the unknowns' order; Z = U^T F.
R5  V: trailing m-k columns of the Householder Q of X = A_ss^{-1} U (LAPACK
    larfg convention); nonsymmetric: V_L from X, V_R from A_ss^{-T} U.
R6  coarse-fill blocks use (U^T A_ss^{-1} U) Z as printed in Eq. (scaling).
R7  degenerate ranks: k = 0 means no fill, E_s = I, the step is a block LU
    step (Sec. 2.2); k = m leaves the cluster untouched for the next level.
R8  eps = 0 is the exact mode: k = m whenever w is non-empty, k = 0 otherwise.
R9  pivot blocks and F_ff are factored by LU without pivoting (Doolittle), the
    nonsymmetric counterpart of the Cholesky factor of Eq. (elim).
R10 the recursion stops at the single root cluster, factored densely.
R11 structural fill a-b for every pair of neighbours of a processed cluster
    is recorded whatever the rank, so patterns do not depend on numbers.
R12 fill whose largest row norm is at most 1e-12 ||A_ss||_F is rounding noise
    of earlier Schur updates (the relative rule of Eq. lra would compress
    noise): it is treated as zero, k = 0 (eps > 0 only).
R14 clusters without a grid: complete recursive bisection of the graph of
    A + A^T to the same depth D; each set is ordered breadth first from a
    pseudo-peripheral vertex (component by component, lowest vertex first,
    neighbours ascending) and its first floor(|S|/2) vertices form the left
    child.
R16 (opt-in, for indefinite systems) A_ss and F_ff are factored with partial
    pivoting, P A = L U: at step j the lowest row at or below j whose |entry|
    is within 1e-10 of the column's largest, rows exchanged across the block.
    The permutation stays inside the cluster, so the stored operators become
    L^{-1} P (and U^{-1}); everything else is unchanged.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg as sla


class Breakdown(RuntimeError):
    """Zero or non-finite pivot in an LU without pivoting."""


# =============================================================== symbolic


@dataclasses.dataclass
class Tree:
    depth: int  # D; levels 0..D, level D is the single root
    nlevels: int
    leaf_dofs: List[np.ndarray]  # DOFs (global ids, ascending) of each leaf = level-0 cluster
    cluster_of_dof: np.ndarray  # level-0 cluster of each DOF
    local_of_dof: np.ndarray  # position of each DOF inside its leaf


def build_tree(dims: Tuple[int, int, int], leaf: int) -> Tree:
    """Reading R1: complete geometric bisection of the grid box (Alg. 1,
    "Partition the graph of A"; the recursive-bisection special case of the
    relation to LoRaSp paragraph)."""
    nx, ny, nz = dims
    n = nx * ny * nz
    depth = 0 if n <= leaf else int(math.ceil(math.log2(n / leaf)))
    boxes = [((0, nx), (0, ny), (0, nz))]
    for _ in range(depth):
        nxt = []
        for b in boxes:
            ext = [b[a][1] - b[a][0] for a in range(3)]
            axis = int(np.argmax(ext))  # first maximum: ties go to x, then y, then z
            lo, hi = b[axis]
            cut = lo + ext[axis] // 2
            left = list(b)
            right = list(b)
            left[axis] = (lo, cut)
            right[axis] = (cut, hi)
            nxt.append(tuple(left))
            nxt.append(tuple(right))
        boxes = nxt
    cluster_of = np.empty(n, dtype=np.int64)
    local_of = np.empty(n, dtype=np.int64)
    leaf_dofs = []
    for c, ((x0, x1), (y0, y1), (z0, z1)) in enumerate(boxes):
        zz, yy, xx = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        ids = np.sort((xx + nx * (yy + ny * zz)).ravel())
        leaf_dofs.append(ids)
        cluster_of[ids] = c
        local_of[ids] = np.arange(ids.size)
    return Tree(depth, depth + 1, leaf_dofs, cluster_of, local_of)


def _level_structure_order(S: np.ndarray, nbrs: List[np.ndarray], inset: np.ndarray) -> List[int]:
    """Reading R14: the vertices of S in breadth-first order from
    pseudo-peripheral roots, one connected component (of the subgraph induced
    by S) after the other, components taken by their lowest vertex.  A root
    search starts at the component's lowest vertex and moves to the lowest
    vertex of the last breadth-first level while that increases the
    eccentricity (at most 8 moves).  Neighbours are visited in ascending
    order."""
    todo = set(int(v) for v in S)
    order: List[int] = []

    def bfs(root):
        seen = {root}
        levels = [[root]]
        while True:
            nxt = []
            for u in levels[-1]:
                for v in nbrs[u]:
                    v = int(v)
                    if inset[v] and v in todo and v not in seen:
                        seen.add(v)
                        nxt.append(v)
            if not nxt:
                return levels
            levels.append(nxt)

    while todo:
        root = min(todo)
        levels = bfs(root)
        for _ in range(8):
            cand = min(levels[-1])
            lv = bfs(cand)
            if len(lv) <= len(levels):
                break
            root, levels = cand, lv
        comp = [v for lev in levels for v in lev]
        order.extend(comp)
        todo.difference_update(comp)
    return order


def build_tree_algebraic(row_ptr: np.ndarray, col_idx: np.ndarray, leaf: int) -> Tree:
    """Reading R14 (Alg. 1 "Partition the graph of A" without a geometry):
    complete recursive bisection of the graph of A + A^T to depth
    D = ceil(log2(N / leaf)); a set goes to two children, the first
    floor(|S| / 2) vertices of its level-structure order to the left one,
    the rest to the right one.  Leaves keep their unknowns in ascending
    order."""
    row_ptr = np.asarray(row_ptr)
    col_idx = np.asarray(col_idx).astype(np.int64)
    n = row_ptr.size - 1
    depth = 0 if n <= leaf else int(math.ceil(math.log2(n / leaf)))
    sets = [set() for _ in range(n)]
    for i in range(n):
        for j in col_idx[row_ptr[i] : row_ptr[i + 1]]:
            j = int(j)
            if j != i:
                sets[i].add(j)
                sets[j].add(i)
    nbrs = [np.array(sorted(x), dtype=np.int64) for x in sets]
    nodes = [np.arange(n)]
    inset = np.zeros(n, dtype=bool)
    for _ in range(depth):
        nxt = []
        for S in nodes:
            inset[:] = False
            inset[S] = True
            order = _level_structure_order(S, nbrs, inset)
            h = len(order) // 2
            nxt.append(np.array(sorted(order[:h]), dtype=np.int64))
            nxt.append(np.array(sorted(order[h:]), dtype=np.int64))
        nodes = nxt
    cluster_of = np.empty(n, dtype=np.int64)
    local_of = np.empty(n, dtype=np.int64)
    for c, ids in enumerate(nodes):
        cluster_of[ids] = c
        local_of[ids] = np.arange(ids.size)
    return Tree(depth, depth + 1, nodes, cluster_of, local_of)


def level0_graph(row_ptr: np.ndarray, col_idx: np.ndarray, cluster_of: np.ndarray, ncl: int) -> List[List[int]]:
    """Neighbour lists of A_B (Eq. quotient) over the leaves, symmetrised,
    from the stored entries of the CSR pattern (reading R2)."""
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    ci = cluster_of[rows]
    cj = cluster_of[col_idx.astype(np.int64)]
    adj = [set() for _ in range(ncl)]
    for a, b in set(zip(ci.tolist(), cj.tolist())):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return [sorted(s) for s in adj]


def greedy_distance2_coloring(adj: Sequence[Sequence[int]]) -> List[int]:
    """Reading R3: clusters at distance <= 2 in A_B get different colours
    (Sec. 2.3: clusters further apart never interact; Sec. 3.4 colouring)."""
    ncl = len(adj)
    color = [-1] * ncl
    for i in range(ncl):
        used = set()
        for j in adj[i]:
            if color[j] >= 0:
                used.add(color[j])
            for l in adj[j]:
                if l != i and color[l] >= 0:
                    used.add(color[l])
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color


def processing_order(color: Sequence[int]) -> List[int]:
    return sorted(range(len(color)), key=lambda i: (color[i], i))


@dataclasses.dataclass
class LevelSymbolic:
    adj: List[List[int]]  # neighbours n(s) at the start of the level
    color: List[int]
    order: List[int]
    pos: List[int]  # processing position of each cluster
    fill: List[List[int]]  # w(s) at the time s is processed, by processing position
    final_pattern: List[List[int]]  # row pattern (incl. diagonal) after the level
    next_adj: List[List[int]]  # neighbour lists of the parent clusters


def simulate_level_pattern(adj: List[List[int]]) -> LevelSymbolic:
    """Structural fill of one level (Sec. 2.3): eliminating s couples every
    pair of its neighbours; w(s) are the clusters coupled to s by such fill
    when s is processed (reading R11 makes this independent of the ranks)."""
    ncl = len(adj)
    color = greedy_distance2_coloring(adj)
    order = processing_order(color)
    pos = [0] * ncl
    for p, s in enumerate(order):
        pos[s] = p
    pattern = [set(adj[i]) | {i} for i in range(ncl)]
    fill = [[] for _ in range(ncl)]
    for s in order:
        nset = set(adj[s])
        w = [t for t in pattern[s] if t != s and t not in nset]
        fill[s] = sorted(w, key=lambda t: pos[t])
        for a in adj[s]:
            pattern[a].update(adj[s])
    final = [sorted(p) for p in pattern]
    npar = (ncl + 1) // 2
    nadj = [set() for _ in range(npar)]
    for a in range(ncl):
        for b in final[a]:
            pa, pb = a // 2, b // 2
            if pa != pb:
                nadj[pa].add(pb)
    return LevelSymbolic(adj, color, order, pos, fill, final, [sorted(s) for s in nadj])


def symbolic_analysis(row_ptr, col_idx, dims, leaf) -> Tuple[Tree, List[LevelSymbolic]]:
    """dims: the grid (nx, ny, nz), or None to partition the graph of A
    (reading R14)."""
    tree = build_tree(dims, leaf) if dims is not None else build_tree_algebraic(row_ptr, col_idx, leaf)
    ncl = len(tree.leaf_dofs)
    adj = level0_graph(row_ptr, col_idx, tree.cluster_of_dof, ncl)
    levels = []
    for lvl in range(tree.nlevels):
        ls = simulate_level_pattern(adj)
        levels.append(ls)
        adj = ls.next_adj
    return tree, levels


# ============================================================ dense kernels


def lu_nopiv(a: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Doolittle LU without pivoting (reading R9): A = L U, L unit lower."""
    n = a.shape[0]
    lu = np.array(a, dtype=np.float64, copy=True)
    for j in range(n):
        p = lu[j, j]
        if p == 0.0 or not np.isfinite(p):
            raise Breakdown(f"pivot {j} of a {n}x{n} block is {p}")
        lu[j + 1 :, j] /= p
        lu[j + 1 :, j + 1 :] -= np.outer(lu[j + 1 :, j], lu[j, j + 1 :])
    return np.tril(lu, -1) + np.eye(n), np.triu(lu)


PIVOT_TIE_LU = 1e-10


def lu_partial(a: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Reading R16: LU with partial pivoting, P A = L U, L unit lower.  At step
    j the pivot is the lowest row at or below j whose |entry| is within
    1e-10 of the column's largest; rows are exchanged across the whole
    matrix.  Returns (L, U, p) with (P A)[i, :] = A[p[i], :]."""
    n = a.shape[0]
    lu = np.array(a, dtype=np.float64, copy=True)
    p = np.arange(n)
    for j in range(n):
        col = np.abs(lu[j:, j])
        mx = col.max() if col.size else 0.0
        if mx == 0.0 or not np.isfinite(mx):
            raise Breakdown(f"pivot {j} of a {n}x{n} block is {mx}")
        i = j + int(np.flatnonzero(col >= (1.0 - PIVOT_TIE_LU) * mx)[0])
        if i != j:
            lu[[j, i], :] = lu[[i, j], :]
            p[[j, i]] = p[[i, j]]
        lu[j + 1 :, j] /= lu[j, j]
        lu[j + 1 :, j + 1 :] -= np.outer(lu[j + 1 :, j], lu[j, j + 1 :])
    return np.tril(lu, -1) + np.eye(n), np.triu(lu), p


def _lsolve(L, B, p=None):
    """L^{-1} P B (P the row permutation p of a pivoted LU; none: identity)."""
    if p is not None:
        B = B[p]
    return sla.solve_triangular(L, B, lower=True, unit_diagonal=True) if L.size else B.copy()


def _usolve(U, B):
    return sla.solve_triangular(U, B, lower=False) if U.size else B.copy()


def _lu_solve(L, U, B, p=None):
    """A^{-1} B with P A = L U."""
    return _usolve(U, _lsolve(L, B, p))


def _lu_solve_t(L, U, B, p=None):
    """A^{-T} B with P A = L U: P^T L^{-T} U^{-T} B."""
    y = sla.solve_triangular(U, B, lower=False, trans="T") if U.size else B.copy()
    y = sla.solve_triangular(L, y, lower=True, unit_diagonal=True, trans="T") if L.size else y
    if p is None:
        return y
    out = np.empty_like(y)
    out[p] = y
    return out


def _right_usolve(B, U):
    """B U^{-1}."""
    if U.size == 0:
        return B.copy()
    return sla.solve_triangular(U, B.T, lower=False, trans="T").T


def _house(x: np.ndarray) -> Tuple[np.ndarray, float, float]:
    """Householder reflector H = I - tau v v^T with v[0] = 1 and H x = beta e_1,
    beta = -sign(alpha) ||x|| (LAPACK larfg convention; tau = 0 when x[1:] = 0)."""
    alpha = float(x[0])
    xnorm = float(np.linalg.norm(x[1:]))
    v = np.zeros_like(x)
    v[0] = 1.0
    if xnorm == 0.0:
        return v, 0.0, alpha
    nrm = math.hypot(alpha, xnorm)
    beta = -nrm if alpha >= 0.0 else nrm
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


PIVOT_TIE_RTOL = 1e-10
FILL_NOISE_FLOOR = 1e-12


def qrcp_truncated(M: np.ndarray, eps: float, fixed_rank: int = 0):
    """Truncated QR with column pivoting of M (rows x cols):
    M[:, piv] = Q R.  Returns (k, R_k, rdiag, piv) with R_k the first k rows of
    R (k x cols, columns in pivot order, rows signed so that R_jj > 0),
    rdiag = |R_jj| of the accepted pivots and piv the full column exchange
    order (accepted pivots first)."""
    rows, n = M.shape
    R = np.array(M, dtype=np.float64, copy=True)
    cols = np.arange(n)
    rdiag: List[float] = []
    r11 = 0.0
    k = 0
    for j in range(min(rows, n)):
        norms2 = np.sum(R[j:, j:] ** 2, axis=0)  # recomputed, not downdated
        mx = float(norms2.max())
        if mx == 0.0:
            break
        p = j + int(np.flatnonzero(norms2 >= (1.0 - PIVOT_TIE_RTOL) * mx)[0])
        rjj = math.sqrt(float(norms2[p - j]))
        if j == 0:
            r11 = rjj
        if rjj <= eps * r11:
            break
        if fixed_rank and j >= fixed_rank:
            break
        R[:, [j, p]] = R[:, [p, j]]
        cols[[j, p]] = cols[[p, j]]
        v, tau, beta = _house(R[j:, j])
        R[j:, j:] -= tau * np.outer(v, v @ R[j:, j:])
        if beta < 0.0:
            R[j, :] = -R[j, :]
        rdiag.append(rjj)
        k = j + 1
    return k, np.triu(R[:k, :]), np.asarray(rdiag), cols


def compress_fill(F: np.ndarray, eps: float, fixed_rank: int = 0):
    """Reading R4 of Eq. (lra): F ~ U Z with U (m x k) orthonormal.

    Returns (k, U, Z, rdiag, piv) with rdiag the |R_jj| of the accepted
    pivots and piv the unknowns of s chosen as pivots."""
    m = F.shape[0]
    k, Rk, rdiag, cols = qrcp_truncated(F.T, eps, fixed_rank)
    if k == 0:
        return 0, np.zeros((m, 0)), np.zeros((0, F.shape[1])), rdiag, cols[:0].copy()
    Mk = np.zeros((m, k))
    Mk[cols, :] = Rk.T  # P R_k^T: row i of R_k^T belongs to unknown cols[i]
    Q, Rq = np.linalg.qr(Mk)
    U = Q * np.where(np.diag(Rq) < 0.0, -1.0, 1.0)[None, :]
    return k, U, U.T @ F, rdiag, cols[:k].copy()


def householder_complement(X: np.ndarray) -> np.ndarray:
    """Reading R5: V = trailing m-k columns of Q = H_1 ... H_k from the
    Householder QR of X (m x k), so that V^T X = 0 and V^T V = I."""
    m, k = X.shape
    R = np.array(X, dtype=np.float64, copy=True)
    Q = np.eye(m)
    for j in range(k):
        v, tau, _ = _house(R[j:, j])
        R[j:, j:] -= tau * np.outer(v, v @ R[j:, j:])
        Q[:, j:] -= tau * np.outer(Q[:, j:] @ v, v)
    return Q[:, k:].copy()


# ============================================================== numeric


@dataclasses.dataclass
class Record:
    """Operator W_s of one cluster (Sec. 2.1)."""

    kind: str  # "empty", "deferred", "full" (E_s = I) or "lowrank"
    m: int
    k: int
    nbrs: List[int]
    nbr_sizes: List[int]  # current sizes of the neighbours when s was processed
    fill: List[int]
    fill_sizes: List[int]
    L: Optional[np.ndarray] = None  # LU of A_ss (P A_ss = L Uu with pivoting)
    Uu: Optional[np.ndarray] = None
    p: Optional[np.ndarray] = None  # row permutation of A_ss's LU (None: unpivoted)
    pf: Optional[np.ndarray] = None  # ... of F_ff's LU
    U: Optional[np.ndarray] = None  # m x k
    Z: Optional[np.ndarray] = None
    VL: Optional[np.ndarray] = None  # m x f
    VR: Optional[np.ndarray] = None
    Lf: Optional[np.ndarray] = None  # LU of F_ff = V_L^T A_ss^{-1} V_R
    Uf: Optional[np.ndarray] = None
    EL: Optional[np.ndarray] = None  # n_tot x f
    ER: Optional[np.ndarray] = None  # f x n_tot
    rdiag: Optional[np.ndarray] = None
    w_tot: int = 0


@dataclasses.dataclass
class Level:
    sym: LevelSymbolic
    m: List[int]  # cluster sizes at the start of the level
    k: List[int]  # sizes after the level (coarse DOFs)
    records: List[Record]
    start_blocks: Optional[Dict[Tuple[int, int], np.ndarray]]
    dofs: Optional[List[Optional[np.ndarray]]]  # original DOFs, while a cluster is still in the original basis
    exec_order: List[int]


@dataclasses.dataclass
class Factor:
    n: int
    symmetric: bool
    eps: float
    tree: Tree
    levels: List[Level]


def _level0_blocks(row_ptr, col_idx, val, tree: Tree) -> Dict[Tuple[int, int], np.ndarray]:
    """Every non-zero block stored densely (Sec. 5.3 notes the implementation
    keeps sparse blocks as dense matrices)."""
    sizes = [d.size for d in tree.leaf_dofs]
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    cols = col_idx.astype(np.int64)
    ci, cj = tree.cluster_of_dof[rows], tree.cluster_of_dof[cols]
    li, lj = tree.local_of_dof[rows], tree.local_of_dof[cols]
    blocks: Dict[Tuple[int, int], np.ndarray] = {}
    for e in range(rows.size):
        key = (int(ci[e]), int(cj[e]))
        b = blocks.get(key)
        if b is None:
            b = blocks[key] = np.zeros((sizes[key[0]], sizes[key[1]]))
        b[li[e], lj[e]] += val[e]
    for c, s in enumerate(sizes):
        if (c, c) not in blocks:
            blocks[(c, c)] = np.zeros((s, s))
    return blocks


def _get(blocks, a, b, cur):
    blk = blocks.get((a, b))
    if blk is None:
        return np.zeros((cur[a], cur[b]))
    return blk


def factor(row_ptr, col_idx, val, dims, leaf: int, eps: float, symmetric: bool,
           fixed_rank: int = 0, keep_blocks: bool = False, progress=None,
           shuffle_within_colors: Optional[np.random.Generator] = None, pivoting: bool = False) -> Factor:
    """Alg. 1 (Hierarchical_Factor) with the low-rank elimination of Sec. 2.1.

    ``shuffle_within_colors`` permutes the execution order of the clusters of
    each colour (Sec. 2.3: clusters more than two apart never interact, so
    the result must not change by a single bit)."""
    row_ptr = np.asarray(row_ptr)
    col_idx = np.asarray(col_idx)
    val = np.asarray(val, dtype=np.float64)
    n = row_ptr.size - 1
    tree, syms = symbolic_analysis(row_ptr, col_idx, dims, leaf)
    blocks = _level0_blocks(row_ptr, col_idx, val, tree)
    cur = [d.size for d in tree.leaf_dofs]
    dofs: Optional[List[Optional[np.ndarray]]] = [d.copy() for d in tree.leaf_dofs]
    levels: List[Level] = []
    for lvl, sym in enumerate(syms):
        m_start = list(cur)
        start = {key: b.copy() for key, b in blocks.items()} if keep_blocks else None
        records: List[Optional[Record]] = [None] * len(cur)
        level_dofs = list(dofs) if dofs is not None else None
        exec_order = list(sym.order)
        if shuffle_within_colors is not None:
            exec_order = []
            for c in range(max(sym.color) + 1):
                grp = [s for s in sym.order if sym.color[s] == c]
                exec_order += [grp[i] for i in shuffle_within_colors.permutation(len(grp))]
        for s in exec_order:
            records[s] = _low_rank_elimination(s, sym, blocks, cur, eps, symmetric, fixed_rank, pivoting)
            if dofs is not None:
                r = records[s]
                if r.kind in ("full", "empty"):
                    dofs[s] = np.zeros(0, dtype=np.int64)
                elif r.kind == "lowrank":
                    dofs[s] = None  # transformed basis
        k_end = list(cur)
        levels.append(Level(sym, m_start, k_end, records, start, level_dofs, exec_order))
        if progress is not None:
            progress(lvl, levels[-1])
        if lvl == len(syms) - 1:
            break
        blocks, cur, dofs = _merge(blocks, cur, dofs, sym)
    return Factor(n, symmetric, eps, tree, levels)


def _low_rank_elimination(s, sym: LevelSymbolic, blocks, cur, eps, symmetric, fixed_rank,
                          pivoting: bool = False) -> Record:
    """LowRank_Elimination of Alg. 1 for cluster s: W_s = P_s G_s E_s."""
    m = cur[s]
    nb = list(sym.adj[s])
    wl = list(sym.fill[s])
    nsz = [cur[a] for a in nb]
    wsz = [cur[t] for t in wl]
    rec = Record("empty", m, 0, nb, nsz, wl, wsz)
    if m == 0:
        return rec
    A_ss = blocks[(s, s)]
    A_sn = np.hstack([_get(blocks, s, a, cur) for a in nb]) if nb else np.zeros((m, 0))
    A_ns = np.vstack([_get(blocks, a, s, cur) for a in nb]) if nb else np.zeros((0, m))
    F_r = np.hstack([_get(blocks, s, t, cur) for t in wl]) if wl else np.zeros((m, 0))
    F = F_r if symmetric else np.hstack([F_r] + [_get(blocks, t, s, cur).T for t in wl])
    rec.w_tot = F_r.shape[1]

    # ---- rank of the fill (Eq. lra)
    if F.shape[1] == 0:
        k, U, Z = 0, None, None
    elif eps == 0.0:
        k, U, Z = m, None, None  # exact mode (reading R8)
    elif np.linalg.norm(F, axis=1).max() <= FILL_NOISE_FLOOR * np.linalg.norm(A_ss):
        k, U, Z = 0, None, None  # reading R12: the fill is rounding noise
    else:
        k, U, Z, rdiag, _ = compress_fill(F, eps, fixed_rank)
        rec.rdiag = rdiag
    rec.k = k
    nt = A_sn.shape[1]

    if k == m:
        rec.kind = "deferred"  # reading R7: nothing eliminated
        return rec

    if pivoting:
        L, Uu, pa = lu_partial(A_ss)  # reading R16
    else:
        (L, Uu), pa = lu_nopiv(A_ss), None
    rec.L, rec.Uu, rec.p = L, Uu, pa
    if k == 0:
        # E_s = I (Sec. 2.2): one block LU step; any fill of s is dropped.
        rec.kind = "full"
        rec.ER = _lsolve(L, A_sn, pa)
        rec.EL = _right_usolve(A_ns, Uu)
        for t in wl:
            blocks[(s, t)] = np.zeros((0, cur[t]))
            blocks[(t, s)] = np.zeros((cur[t], 0))
        for a in nb:
            blocks[(s, a)] = np.zeros((0, cur[a]))
            blocks[(a, s)] = np.zeros((cur[a], 0))
        blocks[(s, s)] = np.zeros((0, 0))
        cur[s] = 0
        _schur(blocks, nb, nsz, rec.EL, rec.ER)
        return rec

    # ---- sparsification operator E_s (Eq. scaling)
    rec.kind = "lowrank"
    Z_r = Z[:, : rec.w_tot]
    Z_c = Z_r if symmetric else Z[:, rec.w_tot :]
    X = _lu_solve(L, Uu, U, pa)  # A_ss^{-1} U
    VL = householder_complement(X)  # V_L^T A_ss^{-1} U = 0
    VR = VL if symmetric else householder_complement(_lu_solve_t(L, Uu, U, pa))
    Ainv_VR = _lu_solve(L, Uu, VR, pa)
    Ainv_Asn = _lu_solve(L, Uu, A_sn, pa)
    F_ff = VL.T @ Ainv_VR  # fine-fine block V^T A_ss^{-1} V
    C = U.T @ X  # coarse-coarse block U^T A_ss^{-1} U
    B_fn = VL.T @ Ainv_Asn  # V^T A_ss^{-1} A_sn
    B_cn = U.T @ Ainv_Asn  # U^T A_ss^{-1} A_sn
    B_nf = A_ns @ Ainv_VR  # A_ns A_ss^{-1} V
    B_nc = A_ns @ X  # A_ns A_ss^{-1} U

    # ---- elimination operator G_s (Eq. elim), F_ff = L_f U_f
    if pivoting:
        Lf, Uf, pf = lu_partial(F_ff)
    else:
        (Lf, Uf), pf = lu_nopiv(F_ff), None
    rec.pf = pf
    ER = _lsolve(Lf, B_fn, pf)  # L_f^{-1} P_f V^T A_ss^{-1} A_sn
    EL = _right_usolve(B_nf, Uf)  # A_ns A_ss^{-1} V U_f^{-1}
    rec.U, rec.Z, rec.VL, rec.VR, rec.Lf, rec.Uf, rec.EL, rec.ER = U, Z, VL, VR, Lf, Uf, EL, ER

    # ---- coarse DOFs of s replace s (permutation P_s, Eq. perm)
    blocks[(s, s)] = C
    off = 0
    for a, sz in zip(nb, nsz):
        blocks[(s, a)] = B_cn[:, off : off + sz].copy()
        blocks[(a, s)] = B_nc[off : off + sz, :].copy()
        off += sz
    off = 0
    for t, sz in zip(wl, wsz):
        blocks[(s, t)] = C @ Z_r[:, off : off + sz]
        blocks[(t, s)] = Z_c[:, off : off + sz].T @ C
        off += sz
    cur[s] = k
    _schur(blocks, nb, nsz, EL, ER)
    assert nt == sum(nsz)
    return rec


def _schur(blocks, nb, nsz, EL, ER):
    """A_nn <- A_nn - E_L E_R for every ordered pair of neighbours (Eq. elim),
    creating the level-1 fill blocks of Sec. 2.3."""
    offs = np.concatenate([[0], np.cumsum(nsz)]).astype(int)
    for i, a in enumerate(nb):
        for j, b in enumerate(nb):
            upd = EL[offs[i] : offs[i + 1], :] @ ER[:, offs[j] : offs[j + 1]]
            blk = blocks.get((a, b))
            if blk is None:
                blocks[(a, b)] = -upd
            else:
                blocks[(a, b)] = blk - upd


def _merge(blocks, cur, dofs, sym: LevelSymbolic):
    """Alg. 1 "Extract A_c": the coarse DOFs of sibling clusters, left then
    right, form the parent cluster of the next level (reading R1)."""
    ncl = len(cur)
    npar = (ncl + 1) // 2
    ch = [[c for c in (2 * p, 2 * p + 1) if c < ncl] for p in range(npar)]
    ncur = [sum(cur[c] for c in ch[p]) for p in range(npar)]
    nblocks: Dict[Tuple[int, int], np.ndarray] = {}
    for p in range(npar):
        for q in set([p] + sym.next_adj[p]):
            blk = np.zeros((ncur[p], ncur[q]))
            r0 = 0
            for a in ch[p]:
                c0 = 0
                for b in ch[q]:
                    sub = blocks.get((a, b))
                    if sub is not None and sub.size:
                        blk[r0 : r0 + cur[a], c0 : c0 + cur[b]] = sub
                    c0 += cur[b]
                r0 += cur[a]
            nblocks[(p, q)] = blk
    ndofs = None
    if dofs is not None and all(d is not None for d in dofs):
        ndofs = [np.concatenate([dofs[c] for c in ch[p]]) for p in range(npar)]
    return nblocks, ncur, ndofs


# ================================================================= solve


def solve(fac: Factor, B: np.ndarray) -> np.ndarray:
    """Alg. 2: forward substitution with W_0 ... W_{m-1} on every level,
    then backward substitution with the transposed operators in reverse."""
    B = np.asarray(B, dtype=np.float64)
    vec1 = B.ndim == 1
    if vec1:
        B = B[:, None]
    tree = fac.tree
    vec = [B[d, :].copy() for d in tree.leaf_dofs]
    fine_all = []
    for li, lev in enumerate(fac.levels):
        fine = [None] * len(vec)
        for s in lev.exec_order:
            fine[s] = _forward(lev.records[s], s, vec)
        fine_all.append(fine)
        if li < len(fac.levels) - 1:
            ncl = len(vec)
            vec = [np.vstack([vec[c] for c in (2 * p, 2 * p + 1) if c < ncl]) for p in range((ncl + 1) // 2)]
    for li in range(len(fac.levels) - 1, -1, -1):
        lev = fac.levels[li]
        if li < len(fac.levels) - 1:
            ncl = len(lev.k)
            child = [None] * ncl
            for p, v in enumerate(vec):
                off = 0
                for c in (2 * p, 2 * p + 1):
                    if c < ncl:
                        child[c] = v[off : off + lev.k[c], :]
                        off += lev.k[c]
            vec = child
        for s in reversed(lev.exec_order):
            _backward(lev.records[s], s, vec, fine_all[li][s])
    X = np.zeros_like(B)
    for c, d in enumerate(tree.leaf_dofs):
        X[d, :] = vec[c]
    return X[:, 0] if vec1 else X


def _forward(rec: Record, s, vec):
    if rec.kind in ("empty", "deferred"):
        return None
    y = vec[s]
    if rec.kind == "full":
        yf = _lsolve(rec.L, y, rec.p)
        vec[s] = np.zeros((0, y.shape[1]))
    else:
        t = _lu_solve(rec.L, rec.Uu, y, rec.p)
        yf = _lsolve(rec.Lf, rec.VL.T @ t, rec.pf)
        vec[s] = rec.U.T @ t
    off = 0
    for a, sz in zip(rec.nbrs, rec.nbr_sizes):
        vec[a] = vec[a] - rec.EL[off : off + sz, :] @ yf
        off += sz
    return yf


def _backward(rec: Record, s, vec, yf):
    if rec.kind in ("empty", "deferred"):
        return
    xn = np.vstack([vec[a] for a in rec.nbrs]) if rec.nbrs else np.zeros((0, yf.shape[1]))
    xf = _usolve(rec.Uf if rec.kind == "lowrank" else rec.Uu, yf - rec.ER @ xn)
    if rec.kind == "full":
        vec[s] = xf
    else:
        vec[s] = _lu_solve(rec.L, rec.Uu, rec.VR @ xf + rec.U @ vec[s], rec.p)


# ================================================================ Krylov


def _csr_mv(row_ptr, col_idx, val, X):
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    out = np.zeros((n, X.shape[1]))
    np.add.at(out, rows, val[:, None] * X[col_idx, :])
    return out


def pcg(row_ptr, col_idx, val, B, precond, tol: float, maxit: int):
    """Preconditioned conjugate gradients, one independent recurrence per
    right-hand side, x0 = 0, stop when ||b - A x|| <= tol ||b|| (Sec. 5.1)."""
    B = np.asarray(B, dtype=np.float64).reshape(B.shape[0], -1)
    nrhs = B.shape[1]
    X = np.zeros_like(B)
    R = B.copy()
    bn = np.linalg.norm(B, axis=0)
    bn[bn == 0] = 1.0
    Zc = precond(R)
    P = Zc.copy()
    rz = np.sum(R * Zc, axis=0)
    active = np.linalg.norm(R, axis=0) > tol * bn
    it = 0
    while active.any() and it < maxit:
        it += 1
        AP = _csr_mv(row_ptr, col_idx, val, P)
        alpha = np.where(active, rz / np.where(active, np.sum(P * AP, axis=0), 1.0), 0.0)
        X += alpha * P
        R -= alpha * AP
        active = active & (np.linalg.norm(R, axis=0) > tol * bn)
        Zc = precond(R)
        rz_new = np.sum(R * Zc, axis=0)
        beta = np.where(active, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
        P = Zc + beta * P
        rz = rz_new
    res = np.linalg.norm(B - _csr_mv(row_ptr, col_idx, val, X), axis=0) / bn
    return X, it, res


def gmres(row_ptr, col_idx, val, b, precond, tol: float, maxit: int, restart: int = 30):
    """Right-preconditioned restarted GMRES with modified Gram-Schmidt, x0 = 0,
    for one right-hand side; stops when the true residual <= tol ||b||."""
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    x = np.zeros(n)
    bn = np.linalg.norm(b) or 1.0
    mv = lambda v: _csr_mv(row_ptr, col_idx, val, v[:, None])[:, 0]
    pc = lambda v: np.asarray(precond(v[:, None]))[:, 0]
    it = 0
    r = b - mv(x)
    while it < maxit and np.linalg.norm(r) > tol * bn:
        beta = np.linalg.norm(r)
        V = np.zeros((n, restart + 1))
        H = np.zeros((restart + 1, restart))
        V[:, 0] = r / beta
        g = np.zeros(restart + 1)
        g[0] = beta
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        j_used = 0
        for j in range(restart):
            it += 1
            w = mv(pc(V[:, j]))
            for i in range(j + 1):
                H[i, j] = w @ V[:, i]
                w -= H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (H[j, j] / den, H[j + 1, j] / den) if den > 0 else (1.0, 0.0)
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_used = j + 1
            if abs(g[j + 1]) <= tol * bn or it >= maxit:
                break
        y = sla.solve_triangular(H[:j_used, :j_used], g[:j_used], lower=False)
        x = x + pc(V[:, :j_used] @ y)
        r = b - mv(x)
    return x, it, np.linalg.norm(r) / bn


# =========================================================== diagnostics


def assemble_level_dense(lev: Level) -> Tuple[np.ndarray, List[int]]:
    """The level's starting matrix as one dense array (clusters in index
    order) and the cluster offsets; needs factor(..., keep_blocks=True)."""
    offs = np.concatenate([[0], np.cumsum(lev.m)]).astype(int)
    a = np.zeros((offs[-1], offs[-1]))
    for (p, q), blk in lev.start_blocks.items():
        if blk.size:
            a[offs[p] : offs[p + 1], offs[q] : offs[q + 1]] = blk
    return a, list(offs)


def factor_flops(fac: Factor) -> float:
    """Algorithmic flops of the factorization from the per-cluster sizes
    (m, k, f, n_tot, w_tot), counted the same way as the GPU library counts."""
    total = 0.0
    for lev in fac.levels:
        for rec in lev.records:
            total += cluster_flops(rec.kind, rec.m, rec.k, sum(rec.nbr_sizes), rec.w_tot, fac.symmetric)
    return total


def cluster_flops(kind: str, m: int, k: int, nt: int, wt: int, symmetric: bool) -> float:
    f = m - k
    if kind in ("empty", "deferred"):
        return 0.0
    fl = 0.0
    ncol = wt if symmetric else 2 * wt
    fl += 2.0 * m ** 3 / 3.0  # LU of the pivot block
    if kind == "full":
        fl += 2.0 * m * m * nt  # E_R and E_L triangular solves
        fl += 2.0 * m * nt * nt  # Schur update
        return fl
    fl += 4.0 * m * ncol * k - 2.0 * k * k * (m + ncol) + 4.0 * k ** 3 / 3.0  # QRCP
    fl += 2.0 * m * k * ncol  # Z
    fl += 2.0 * m * m * k * (1 if symmetric else 2)  # X
    fl += 4.0 * m * k * f * (1 if symmetric else 2)  # complements
    fl += 2.0 * m * m * f  # A^{-1} V
    fl += 2.0 * m * f * f + 2.0 * f ** 3 / 3.0  # F_ff and its LU
    fl += 2.0 * m * m * nt  # A^{-1} A_sn
    fl += 2.0 * m * nt * (k + f) * 2  # B_fn, B_cn, B_nf, B_nc
    fl += 2.0 * f * f * nt  # E_R, E_L triangular solves
    fl += 2.0 * m * k * k + 2.0 * k * k * wt * (1 if symmetric else 2)  # C, C Z
    fl += 2.0 * f * nt * nt  # Schur update
    return fl
