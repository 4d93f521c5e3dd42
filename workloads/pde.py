"""Synthetic PDE-shaped sparse systems on lexicographic grids.

Conventions shared by every generator:

* unknown (x, y, z) of an nx-by-ny-by-nz grid has index x + nx*(y + ny*z)
  (x fastest); 2D grids have nz = 1, 1D grids ny = nz = 1;
* Dirichlet boundaries (couplings that would leave the grid are dropped);
* CSR with int64 row pointers, int32 column indices sorted ascending within a
  row, float64 values;
* right-hand sides are uniform on [-1, 1) from ``numpy.random.default_rng``,
  stored column-major (shape (n, nrhs), Fortran order).

The paper evaluates on 3D Poisson / variable-coefficient Poisson / Helmholtz
model problems (Sec. 5.1) and on SuiteSparse matrices (Table 1); the
generators below stand in for those with seeded synthetic systems of the same
stencil shapes.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int64, n+1
    col_idx: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        a[rows, self.col_idx] = self.val
        return a

    def matvec(self, x: np.ndarray) -> np.ndarray:
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        if x.ndim == 1:
            return np.bincount(rows, weights=self.val * x[self.col_idx], minlength=self.n)
        out = np.zeros((self.n, x.shape[1]))
        np.add.at(out, rows, self.val[:, None] * x[self.col_idx])
        return out

    def is_symmetric(self) -> bool:
        d = self.to_dense() if self.n <= 4096 else None
        if d is not None:
            return bool(np.array_equal(d, d.T))
        import scipy.sparse as sp

        m = sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))
        return (abs(m - m.T)).nnz == 0


@dataclasses.dataclass
class Problem:
    name: str
    A: CSR
    dims: Tuple[int, int, int]  # (nx, ny, nz)
    dim: int  # 1, 2 or 3
    B: np.ndarray  # (n, nrhs) float64, Fortran order
    eps: float
    leaf: int
    tol: float
    symmetric: bool
    krylov: str  # "direct", "pcg" or "gmres"


def _coo_to_csr(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr, cols.astype(np.int32), vals.astype(np.float64))


def _grid_ids(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def _stencil_csr(nx, ny, nz, diag, offs):
    """diag: (n,) values; offs: list of ((dx,dy,dz), coeff array (n,)) for the
    coupling of unknown i to its neighbour at offset (dx,dy,dz)."""
    n = nx * ny * nz
    x, y, z = _grid_ids(nx, ny, nz)
    idx = np.arange(n)
    rows = [idx]
    cols = [idx]
    vals = [np.asarray(diag, dtype=np.float64)]
    for (dx, dy, dz), c in offs:
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
        rows.append(idx[ok])
        cols.append(idx[ok] + dx + nx * (dy + ny * dz))
        vals.append(np.broadcast_to(np.asarray(c, dtype=np.float64), (n,))[ok])
    return _coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def chain1d(n: int) -> CSR:
    """1D Dirichlet Laplacian: 2 on the diagonal, -1 off it."""
    return _stencil_csr(n, 1, 1, np.full(n, 2.0), [((-1, 0, 0), -1.0), ((1, 0, 0), -1.0)])


def poisson2d(nx: int, ny: int) -> CSR:
    """5-point Laplacian, 4 on the diagonal, -1 to each grid neighbour."""
    n = nx * ny
    offs = [((-1, 0, 0), -1.0), ((1, 0, 0), -1.0), ((0, -1, 0), -1.0), ((0, 1, 0), -1.0)]
    return _stencil_csr(nx, ny, 1, np.full(n, 4.0), offs)


def poisson3d(nx: int, ny: int, nz: int) -> CSR:
    """7-point Laplacian, 6 on the diagonal, -1 to each grid neighbour."""
    n = nx * ny * nz
    offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    return _stencil_csr(nx, ny, nz, np.full(n, 6.0), [(o, -1.0) for o in offs])


def gaussian_field3d(rng: np.random.Generator, nx: int, ny: int, nz: int, corr_len: float, sigma: float) -> np.ndarray:
    """Seeded smooth Gaussian field on cell centres, shape (nz, ny, nx).

    White N(0,1) noise is convolved with a separable Gaussian kernel of
    standard deviation corr_len/sqrt(2) cells (truncated at 3 standard
    deviations, zero padding), then scaled to standard deviation ``sigma``.
    """
    white = rng.standard_normal((nz, ny, nx))
    s = corr_len / math.sqrt(2.0)
    r = int(math.ceil(3.0 * s))
    t = np.arange(-r, r + 1, dtype=np.float64)
    ker = np.exp(-0.5 * (t / s) ** 2)
    ker /= ker.sum()
    g = white
    # centred part of the full convolution: the grid keeps its size also when
    # the kernel is longer than a side
    for axis in range(3):
        g = np.apply_along_axis(lambda v: np.convolve(v, ker, mode="full")[r : r + v.size], axis, g)
    g = g - g.mean()
    return sigma * g / g.std()


def diffusion3d_from_coeff(a: np.ndarray) -> CSR:
    """Cell-centred finite-volume 7-point diffusion on a (nz,ny,nx) grid with
    cell coefficients ``a``: interior face transmissibility 2 a_i a_j/(a_i+a_j),
    Dirichlet boundary face 2 a_i; row sum of off-diagonals = -diag + boundary
    terms (an SPD M-matrix)."""
    nz, ny, nx = a.shape
    af = a.ravel()
    n = af.size
    x, y, z = _grid_ids(nx, ny, nz)
    diag = np.zeros(n)
    offs = []
    for (dx, dy, dz) in [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]:
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
        j = np.where(ok, np.arange(n) + dx + nx * (dy + ny * dz), 0)
        aj = af[j]
        t = np.where(ok, 2.0 * af * aj / (af + aj), 2.0 * af)
        diag += t
        offs.append(((dx, dy, dz), -t))
    return _stencil_csr(nx, ny, nz, diag, offs)


def diffusion3d_expgauss(rng: np.random.Generator, side: int, sigma: float = 2.0, corr_len: float = 8.0) -> CSR:
    g = gaussian_field3d(rng, side, side, side, corr_len, sigma)
    return diffusion3d_from_coeff(np.exp(g))


def quantized_field3d(rng: np.random.Generator, nx: int, ny: int, nz: int, dev_cells: float = 4.0,
                      high: float = 1e2, low: float = 1e-2) -> np.ndarray:
    """The quantized high-contrast random field of the paper's variable-
    coefficient Poisson test (Sec. 5.1), shape (nz, ny, nx): uniform [0, 1)
    noise on the cells, convolved with a Gaussian of standard deviation
    dev_cells cells (4h), then set to ``high`` where it exceeds 0.5 and to
    ``low`` elsewhere.  The kernel is separable, truncated at 3 standard
    deviations, and normalised by its weight inside the grid at every cell
    (near the boundary the average is taken over the cells that exist, so the
    field keeps mean 0.5 and the split stays even)."""
    u = rng.uniform(0.0, 1.0, (nz, ny, nx))
    r = int(math.ceil(3.0 * dev_cells))
    t = np.arange(-r, r + 1, dtype=np.float64)
    ker = np.exp(-0.5 * (t / dev_cells) ** 2)

    def conv(v):
        return np.convolve(v, ker, mode="full")[r : r + v.size]

    g, w = u, np.ones_like(u)
    for axis in range(3):
        g = np.apply_along_axis(conv, axis, g)
        w = np.apply_along_axis(conv, axis, w)
    g = g / w
    return np.where(g > 0.5, high, low)


def vc_poisson3d(rng: np.random.Generator, side: int, dev_cells: float = 4.0) -> CSR:
    """Variable-coefficient Poisson -div(a grad u) on a side^3 grid with the
    quantized high-contrast field a (values 1e2 / 1e-2, Sec. 5.1), 7-point
    finite-volume stencil with harmonic face averages."""
    return diffusion3d_from_coeff(quantized_field3d(rng, side, side, side, dev_cells))


def helmholtz3d(side: int, points_per_wavelength: float = 32.0) -> CSR:
    """The paper's third test problem (Sec. 5.1): (-Laplace - k^2) u on a
    side^3 grid of the unit cube, 7-point stencil with Dirichlet boundaries,
    scaled by h^2: 6 - (k h)^2 on the diagonal and -1 to each neighbour.  The
    resolution is fixed, k h = 2 pi / points_per_wavelength (32 in the paper),
    so the wave number grows with the grid: with unit wave speed, side = 32 f
    for the frequency f (1 Hz at 32^3, 4 Hz at 128^3).  Symmetric and
    indefinite once (k h)^2 exceeds the smallest Laplacian eigenvalue."""
    n = side ** 3
    kh2 = (2.0 * math.pi / points_per_wavelength) ** 2
    offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    return _stencil_csr(side, side, side, np.full(n, 6.0 - kh2), [(o, -1.0) for o in offs])


def zero_diagonal_grid2d(rng: np.random.Generator, nx: int, ny: int) -> CSR:
    """A symmetric indefinite matrix whose diagonal is zero: the 5-point grid
    graph with random weights, a_ij = a_ji = -w_ij, w_ij uniform [0.5, 1.5).
    LU without pivoting fails at the first step of every block; with partial
    pivoting a block is singular only if its subgraph is (e.g. an odd number
    of cells of a bipartite grid)."""
    A = poisson2d(nx, ny)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    cols = A.col_idx.astype(np.int64)
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    uniq, inv = np.unique(lo * A.n + hi, return_inverse=True)
    w = rng.uniform(0.5, 1.5, uniq.size)[inv]
    return CSR(A.n, A.row_ptr, A.col_idx, np.where(rows == cols, 0.0, -w))


def random_geometric_spd(rng: np.random.Generator, n: int, degree: float = 8.0, shift: float = 0.05,
                         nonsym: float = 0.0) -> CSR:
    """An unstructured sparse matrix with no grid: n random points in the unit
    square, numbered in random order, coupled when closer than the radius
    that gives about ``degree`` neighbours each; weights w_ij = 1 + u_ij
    (u_ij uniform [0, 1)).  The matrix is the weighted graph Laplacian plus
    ``shift`` times its diagonal (symmetric positive definite); with
    nonsym > 0 every coupling a_ij is scaled by (1 + nonsym v_ij), v_ij
    uniform [-1, 1) drawn per direction (then diagonally dominant by rows)."""
    pts = rng.uniform(0.0, 1.0, (n, 2))
    r = math.sqrt(degree / (math.pi * n))
    cell = np.floor(pts / r).astype(np.int64)
    ncell = int(math.ceil(1.0 / r)) + 1
    key = cell[:, 0] * ncell + cell[:, 1]
    order = np.argsort(key, kind="stable")
    rows, cols = [], []
    buckets = {}
    for i in order:
        buckets.setdefault(int(key[i]), []).append(int(i))
    for i in range(n):
        cx, cy = cell[i]
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for j in buckets.get(int((cx + dx) * ncell + (cy + dy)), ()):
                    if j > i and np.sum((pts[i] - pts[j]) ** 2) < r * r:
                        rows.append(i)
                        cols.append(j)
    rows = np.array(rows, dtype=np.int64)
    cols = np.array(cols, dtype=np.int64)
    w = 1.0 + rng.uniform(0.0, 1.0, rows.size)
    R = np.concatenate([rows, cols])
    C = np.concatenate([cols, rows])
    V = -np.concatenate([w, w])
    if nonsym > 0:
        V = V * (1.0 + nonsym * rng.uniform(-1.0, 1.0, V.size))
    diag = np.zeros(n)
    np.add.at(diag, R, -V)
    diag = diag * (1.0 + shift) + shift
    R = np.concatenate([R, np.arange(n)])
    C = np.concatenate([C, np.arange(n)])
    V = np.concatenate([V, diag])
    return _coo_to_csr(n, R, C, V)


def convdiff2d_upwind(side: int, peclet: float, theta: float) -> CSR:
    """-Laplace(u) + b.grad(u) on the unit square, first-order upwind, h = 1/(side+1),
    b = Pe (cos theta, sin theta), scaled by h^2 (nonsymmetric, diagonally dominant)."""
    h = 1.0 / (side + 1)
    bx, by = peclet * math.cos(theta), peclet * math.sin(theta)
    n = side * side
    diag = np.full(n, 4.0 + h * (abs(bx) + abs(by)))
    offs = [
        ((-1, 0, 0), -1.0 - h * max(bx, 0.0)),
        ((1, 0, 0), -1.0 - h * max(-bx, 0.0)),
        ((0, -1, 0), -1.0 - h * max(by, 0.0)),
        ((0, 1, 0), -1.0 - h * max(-by, 0.0)),
    ]
    return _stencil_csr(side, side, 1, diag, offs)


def random_spd_blocks(rng: np.random.Generator, nx: int, ny: int, nz: int = 1, shift: float = 0.05) -> CSR:
    """Random-weight grid-graph Laplacian plus a small diagonal shift (SPD
    M-matrix) on a 2D/3D grid: edge weights uniform on [0.1, 10)."""
    n = nx * ny * nz
    x, y, z = _grid_ids(nx, ny, nz)
    idx = np.arange(n)
    rows, cols, vals = [], [], []
    diag = np.full(n, shift)
    dirs = [(1, 0, 0), (0, 1, 0)] + ([(0, 0, 1)] if nz > 1 else [])
    for (dx, dy, dz) in dirs:
        ok = (x + dx < nx) & (y + dy < ny) & (z + dz < nz)
        i = idx[ok]
        j = i + dx + nx * (dy + ny * dz)
        wgt = rng.uniform(0.1, 10.0, size=i.size)
        rows += [i, j]
        cols += [j, i]
        vals += [-wgt, -wgt]
        np.add.at(diag, i, wgt)
        np.add.at(diag, j, wgt)
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    return _coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def one_sided_dd(rng: np.random.Generator, nx: int, ny: int, drop: float = 0.35, far: float = 0.06) -> CSR:
    """Structurally nonsymmetric 2D grid operator: each 5-point coupling is
    kept with probability 1 - drop on its own (so (i, j) often has no (j, i)),
    and a fraction `far` of the rows gains one coupling to a uniformly chosen
    unknown.  Off-diagonals uniform on (-1, 0]; diagonal = 1.5 * max(row sum,
    column sum) + 0.1, so the matrix is diagonally dominant by rows and
    columns."""
    n = nx * ny
    x, y, _ = _grid_ids(nx, ny, 1)
    idx = np.arange(n)
    rows, cols = [], []
    for (dx, dy) in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
        i = idx[ok]
        i = i[rng.uniform(size=i.size) >= drop]
        rows.append(i)
        cols.append(i + dx + nx * dy)
    fr = idx[rng.uniform(size=n) < far]
    fc = rng.integers(0, n, size=fr.size)
    keep = fc != fr
    rows.append(fr[keep])
    cols.append(fc[keep])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    pair = np.unique(r.astype(np.int64) * n + c)  # a far coupling may repeat a grid one
    r, c = pair // n, pair % n
    v = -rng.uniform(0.0, 1.0, size=r.size)
    rsum = np.zeros(n)
    csum = np.zeros(n)
    np.add.at(rsum, r, -v)
    np.add.at(csum, c, -v)
    r = np.concatenate([r, idx])
    c = np.concatenate([c, idx])
    v = np.concatenate([v, 1.5 * np.maximum(rsum, csum) + 0.1])
    return _coo_to_csr(n, r, c, v)


def random_nonsym_dd(rng: np.random.Generator, nx: int, ny: int, nz: int = 1) -> CSR:
    """Random nonsymmetric grid operator with positive diagonal dominance:
    off-diagonals uniform on (-2, 0], diagonal = 1.2 * max(row, column) sum."""
    n = nx * ny * nz
    x, y, z = _grid_ids(nx, ny, nz)
    idx = np.arange(n)
    rows, cols, vals = [], [], []
    rsum = np.zeros(n)
    csum = np.zeros(n)
    dirs = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0)] + ([(0, 0, 1), (0, 0, -1)] if nz > 1 else [])
    for (dx, dy, dz) in dirs:
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
        i = idx[ok]
        j = i + dx + nx * (dy + ny * dz)
        v = -rng.uniform(0.0, 2.0, size=i.size)
        rows.append(i)
        cols.append(j)
        vals.append(v)
        np.add.at(rsum, i, -v)
        np.add.at(csum, j, -v)
    rows.append(idx)
    cols.append(idx)
    vals.append(1.2 * np.maximum(rsum, csum) + 0.1)
    return _coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def rhs_uniform(rng: np.random.Generator, n: int, nrhs: int) -> np.ndarray:
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(nrhs, n)).T)


# ---------------------------------------------------------------- configs


def config1(seed: int = 1) -> Problem:
    """2D 5-point Poisson 32x32, leaves of 16, eps 1e-6, one RHS, direct solve."""
    rng = np.random.default_rng(seed)
    A = poisson2d(32, 32)
    return Problem("poisson2d_32", A, (32, 32, 1), 2, rhs_uniform(rng, A.n, 1), 1e-6, 16, 0.0, True, "direct")


def config2(seed: int = 2, side: int = 64, nrhs: int = 8) -> Problem:
    """3D 7-point Poisson side^3 (64^3 by default), leaves of 64, eps 1e-4,
    used as CG preconditioner for 8 RHS to relative residual 1e-10."""
    rng = np.random.default_rng(seed)
    A = poisson3d(side, side, side)
    return Problem(f"poisson3d_{side}", A, (side, side, side), 3, rhs_uniform(rng, A.n, nrhs), 1e-4, 64, 1e-10, True, "pcg")


def config3(seed: int = 3, side: int = 128, nrhs: int = 1) -> Problem:
    """3D variable-coefficient diffusion, coefficients exp(g) with g a Gaussian
    field of standard deviation 2 and correlation length 8 cells; eps 1e-3."""
    rng = np.random.default_rng(seed)
    A = diffusion3d_expgauss(rng, side, 2.0, 8.0)
    return Problem(f"diffusion3d_expgauss_{side}", A, (side, side, side), 3, rhs_uniform(rng, A.n, nrhs), 1e-3, 64, 1e-10, True, "pcg")


def config4_batch(seed: int = 4, count: int = 256, side_lo: int = 64, side_hi: int = 512) -> List[Problem]:
    """Batch of independent 2D upwind convection-diffusion systems: side uniform
    in [side_lo, side_hi], Peclet uniform in [1, 100], direction uniform."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=count)
    pes = rng.uniform(1.0, 100.0, size=count)
    thetas = rng.uniform(0.0, 2.0 * math.pi, size=count)
    out = []
    for i in range(count):
        A = convdiff2d_upwind(int(sides[i]), float(pes[i]), float(thetas[i]))
        s = int(sides[i])
        out.append(Problem(f"convdiff2d_{s}_{i}", A, (s, s, 1), 2, rhs_uniform(rng, A.n, 1), 1e-3, 64, 1e-10, False, "gmres"))
    return out


def make_config(i: int, seed: Optional[int] = None, **kw):
    seed = i if seed is None else seed
    return {1: config1, 2: config2, 3: config3, 4: config4_batch}[i](seed, **kw)


@dataclasses.dataclass
class Request:
    t_arrival: float
    op_key: int
    kind: str  # "diff3d" or "convdiff2d"
    side: int
    param: Tuple[float, ...]
    nrhs: int
    rhs_seed: int


def serving_stream(seed: int, n_requests: int, rate: float, reuse: float = 0.3,
                   side3d: Tuple[int, int] = (32, 96), side2d: Tuple[int, int] = (256, 1024)) -> List[Request]:
    """Poisson arrivals (rate per second) of solve requests: 60% 3D lognormal
    diffusion operators, 40% 2D convection-diffusion operators, 1-16 RHS each;
    with probability ``reuse`` a request names a uniformly chosen earlier
    operator key instead of a new one."""
    rng = np.random.default_rng(seed)
    t = 0.0
    ops: List[Tuple[int, str, int, Tuple[float, ...]]] = []
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        nrhs = int(rng.integers(1, 17))
        if ops and rng.uniform() < reuse:
            key, kind, side, param = ops[int(rng.integers(0, len(ops)))]
        else:
            key = len(ops)
            if rng.uniform() < 0.6:
                kind, side = "diff3d", int(rng.integers(side3d[0], side3d[1] + 1))
                param = (float(rng.integers(0, 2**31 - 1)),)
            else:
                kind, side = "convdiff2d", int(rng.integers(side2d[0], side2d[1] + 1))
                param = (float(rng.uniform(1.0, 100.0)), float(rng.uniform(0.0, 2.0 * math.pi)))
            ops.append((key, kind, side, param))
        out.append(Request(t, key, kind, side, param, nrhs, int(rng.integers(0, 2**31 - 1))))
    return out


def build_request_operator(req: Request) -> Tuple[CSR, Tuple[int, int, int], int, bool]:
    """Matrix, grid dims, dimension and symmetry flag of a serving request."""
    if req.kind == "diff3d":
        rng = np.random.default_rng(int(req.param[0]))
        g = gaussian_field3d(rng, req.side, req.side, req.side, 8.0, 1.5)
        return diffusion3d_from_coeff(np.exp(g)), (req.side,) * 3, 3, True
    A = convdiff2d_upwind(req.side, req.param[0], req.param[1])
    return A, (req.side, req.side, 1), 2, False
