"""Seeded input generators (no GPU): sizes, symmetry and the statistics the
workloads are specified by."""

import math

import numpy as np
import scipy.sparse as sp

from workloads import (config4_batch, convdiff2d_upwind, diffusion3d_from_coeff, gaussian_field3d, serving_stream,
                       build_request_operator, one_sided_dd)


def _csr(A):
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))


def test_gaussian_field_keeps_grid_size_and_sigma():
    """Sides below the kernel length (2 ceil(3 * 8 / sqrt 2) + 1 = 35) keep
    their size; standard deviation is the requested sigma; on a side above
    the kernel length each axis pass equals numpy's centred convolution."""
    for n in (8, 20, 34, 35, 48):
        g = gaussian_field3d(np.random.default_rng(1), n, n + 1, n + 2, 8.0, 1.5)
        assert g.shape == (n + 2, n + 1, n)
        assert abs(g.std() - 1.5) < 1e-12 and abs(g.mean()) < 1e-12
    s = 8.0 / math.sqrt(2.0)
    r = int(math.ceil(3 * s))
    t = np.arange(-r, r + 1, dtype=float)
    ker = np.exp(-0.5 * (t / s) ** 2)
    ker /= ker.sum()
    v = np.random.default_rng(2).standard_normal(50)
    assert np.allclose(np.convolve(v, ker, mode="full")[r : r + 50], np.convolve(v, ker, mode="same"))


def test_diffusion_operator_is_spd_m_matrix():
    a = np.exp(gaussian_field3d(np.random.default_rng(3), 6, 5, 4, 8.0, 2.0))
    A = _csr(diffusion3d_from_coeff(a)).toarray()
    assert A.shape == (120, 120)
    assert np.allclose(A, A.T)
    assert np.all(np.diag(A) > 0) and np.all(A - np.diag(np.diag(A)) <= 0)
    assert np.linalg.eigvalsh(A).min() > 0


def test_convdiff_upwind_row_sums_and_nonsymmetry():
    A = _csr(convdiff2d_upwind(10, 50.0, 0.7)).toarray()
    assert not np.allclose(A, A.T)
    # interior rows sum to zero (consistent discretisation of -Lap + b.grad)
    interior = [i + 10 * j for i in range(1, 9) for j in range(1, 9)]
    assert np.allclose(A[interior].sum(axis=1), 0.0)
    assert np.all(np.diag(A) >= np.abs(A - np.diag(np.diag(A))).sum(axis=1) - 1e-12)


def test_one_sided_operator_pattern_and_dominance():
    """Sorted, duplicate-free rows; couplings without their transpose; strict
    diagonal dominance by rows and by columns."""
    C = one_sided_dd(np.random.default_rng(7), 29, 22)
    for i in range(C.n):
        row = C.col_idx[C.row_ptr[i]:C.row_ptr[i + 1]]
        assert np.all(np.diff(row) > 0)
    A = _csr(C).toarray()
    S = A != 0
    assert (S & ~S.T).sum() > 0
    off = np.abs(A - np.diag(np.diag(A)))
    assert np.all(np.diag(A) > off.sum(axis=1)) and np.all(np.diag(A) > off.sum(axis=0))


def test_batch_workload_ranges():
    probs = config4_batch(count=64)
    sides = np.array([p.dims[0] for p in probs])
    assert len(probs) == 64 and sides.min() >= 64 and sides.max() <= 512
    assert all(p.A.n == p.dims[0] * p.dims[1] for p in probs)
    assert all(p.B.shape == (p.A.n, 1) for p in probs)


def test_serving_stream_mix_and_reuse():
    reqs = serving_stream(5, 2000, rate=10.0)
    t = np.array([r.t_arrival for r in reqs])
    assert np.all(np.diff(t) > 0) and abs(np.mean(np.diff(t)) - 0.1) < 0.01
    keys = [r.op_key for r in reqs]
    reuse = 1 - len(set(keys)) / len(keys)
    assert 0.25 < reuse < 0.35
    new = {}
    for r in reqs:
        new.setdefault(r.op_key, r)
    frac3d = np.mean([r.kind == "diff3d" for r in new.values()])
    assert 0.55 < frac3d < 0.65
    assert all(1 <= r.nrhs <= 16 for r in reqs)
    small = [r for r in new.values() if r.kind == "diff3d"][:2] + [r for r in new.values() if r.kind == "convdiff2d"][:1]
    for r in small:
        r.side = min(r.side, 24)  # keep the check cheap
        A, dims, dim, sym = build_request_operator(r)
        assert A.n == int(np.prod(dims)) and sym == (r.kind == "diff3d")


def test_quantized_high_contrast_field():
    """Sec. 5.1's field: two values, an even split, spatially correlated at
    the 4-cell scale, seeded; one cell checked against a brute-force
    normalised Gaussian average of the same uniform draws."""
    from workloads import quantized_field3d

    rng = np.random.default_rng(1)
    a = quantized_field3d(rng, 20, 18, 16)
    assert a.shape == (16, 18, 20)
    assert set(np.unique(a)) == {1e-2, 1e2}
    assert 0.35 < (a > 1).mean() < 0.65
    assert (a[:, :, 1:] == a[:, :, :-1]).mean() > 0.85  # neighbours mostly agree
    assert np.array_equal(a, quantized_field3d(np.random.default_rng(1), 20, 18, 16))
    u = np.random.default_rng(1).uniform(0.0, 1.0, (16, 18, 20))
    z, y, x = np.meshgrid(np.arange(16), np.arange(18), np.arange(20), indexing="ij")
    for (k, j, i) in [(8, 9, 10), (0, 0, 0), (15, 3, 19)]:
        d = np.maximum.reduce([np.abs(x - i), np.abs(y - j), np.abs(z - k)])
        w = np.exp(-0.5 * (((x - i) / 4.0) ** 2 + ((y - j) / 4.0) ** 2 + ((z - k) / 4.0) ** 2)) * (d <= 12)
        avg = (w * u).sum() / w.sum()
        if abs(avg - 0.5) > 1e-9:
            assert (a[k, j, i] > 1) == (avg > 0.5)


def test_vc_poisson_is_spd_m_matrix():
    from workloads import vc_poisson3d

    A = vc_poisson3d(np.random.default_rng(2), 6)
    D = A.to_dense()
    assert np.array_equal(D, D.T)
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 0)
    assert np.all(np.diag(D) >= -off.sum(axis=1) - 1e-12)
    assert np.linalg.eigvalsh(D).min() > 0


def test_helmholtz_negative_eigenvalues_closed_form():
    """The Dirichlet 7-point Laplacian on n^3 has the eigenvalues
    sum_d 4 sin^2(pi i_d / (2 (n + 1))), i_d = 1..n; the Helmholtz matrix
    shifts them by -(2 pi / ppw)^2, so its negative eigenvalues are counted
    in closed form.  Checked against a dense eigensolver (inertia), with the
    diagonal, the couplings and the symmetry."""
    from workloads import helmholtz3d

    for side, ppw in ((8, 4.0), (10, 6.0), (12, 8.0)):
        A = helmholtz3d(side, ppw)
        D = A.to_dense()
        assert np.allclose(D, D.T)
        kh2 = (2 * np.pi / ppw) ** 2
        assert np.allclose(np.diag(D), 6.0 - kh2)
        off = D - np.diag(np.diag(D))
        assert set(np.unique(off)) <= {0.0, -1.0} and np.all((off != 0).sum(axis=1) <= 6)
        lam1 = 4 * np.sin(np.pi * np.arange(1, side + 1) / (2 * (side + 1))) ** 2
        lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
        neg = int(np.sum(lam < kh2))
        assert neg > 0
        assert int(np.sum(np.linalg.eigvalsh(D) < 0)) == neg
    # the paper's resolution: 32 points per wavelength, 1 Hz on 32^3
    A = helmholtz3d(32)
    assert A.n == 32 ** 3 and np.isclose(A.val[A.col_idx == np.repeat(np.arange(A.n), np.diff(A.row_ptr))][0],
                                         6.0 - (2 * np.pi / 32) ** 2)
