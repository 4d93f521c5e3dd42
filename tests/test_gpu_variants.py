"""Every kernel variant of the factorization compared with the CPU oracle,
element by element, through the C ABI.

Two routes reach the variants that production picks by size:
  * inputs with large leaves, which reach them the way full-size problems
    do (clusters above 128 and 192 unknowns, coarse sizes above 64, complete
    levels wider than one 128-column panel);
  * hs_config_set, which lowers the size thresholds so that the same
    production code paths run on inputs small enough for the oracle (a Gram
    workgroup that sums several fill partners, Schur tiles without the LDS
    pointer table or offsets, the memory-resident pivot kernel, the per-wave
    triangular inverses, the in-memory Householder complement, Q without the
    WY form, U by Householder QR, narrow dense panels).

Bars are those of parity_util: sizes and ranks bit-exact, level matrices and
stored operators within 1e-10 relative at eps = 0 (tol_eps(eps) and
100 tol_eps(eps) at eps > 0), solves within 1e-8.
"""

import numpy as np
import pytest

from parity_util import compare_factor, fill_ratio_of_c1, knobs, scaled_coupling_poisson, solve_both
from workloads import convdiff2d_upwind, poisson2d, poisson3d, random_nonsym_dd

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


def _check_solve(P, fo, F, A):
    B, Xo, Xg = solve_both(P, torch, fo, F, A.n)
    err = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    assert err < 1e-8, err
    return err


# ---------------------------------------------------------------- large leaves
# (name, matrix, dims, leaf, eps, symmetric, what the oracle must show)
LARGE = [
    # level 0: clusters of 144 > 128 with fill at eps > 0 -> pivot kernel with
    # its working matrix in memory, right-looking pivoted Cholesky, complement
    # QR in memory, 12-block triangular inverses (128 < m <= 192)
    ("p2d_leaf144", lambda: poisson2d(48, 48), (48, 48, 1), 144, 1e-4, True, dict(max_lowrank_m=144)),
    # clusters of 256 > 192: per-wave triangular inverses
    ("p2d_leaf256", lambda: poisson2d(64, 64), (64, 64, 1), 256, 1e-4, True, dict(max_lowrank_m=256)),
    # coarse sizes above 64 (k = 65 at m = 108): complement QR in memory at
    # m <= 128; two-slot register QR for 64 < m <= 128 with k <= 64
    ("p3d_leaf200", lambda: poisson3d(12, 12, 12), (12, 12, 12), 200, 1e-4, True, dict(max_k=65)),
    # exact mode: block LU steps of clusters up to 216 (per-wave inverses in the
    # memory-resident pivot kernel), complete level of 1080 unknowns factored
    # with 9 dense panels, its clusters of up to 324 inverted per wave
    ("p3d_leaf160_exact", lambda: poisson3d(12, 12, 12), (12, 12, 12), 160, 0.0, True, dict(max_m=324)),
    # nonsymmetric with clusters of 144: both complements, row and column fill
    ("convdiff_leaf144", lambda: convdiff2d_upwind(48, 50.0, 0.3), (48, 48, 1), 144, 1e-4, False,
     dict(max_lowrank_m=144)),
]


@pytest.mark.parametrize("name,mk,dims,leaf,eps,sym,expect", LARGE, ids=[c[0] for c in LARGE])
def test_large_clusters(P, name, mk, dims, leaf, eps, sym, expect):
    A = mk()
    print(f"[variants] {name}: n={A.n} leaf={leaf} eps={eps}", flush=True)
    fo, F, st = compare_factor(P, A, dims, leaf, eps, sym)
    for key, val in expect.items():
        assert st[key] >= val, (key, st[key], val)
    err = _check_solve(P, fo, F, A)
    print(f"[variants] {name}: {st} solve {err:.2e}", flush=True)


# ------------------------------------------------------- thresholds lowered
SMALL = {
    "p3d": (lambda: poisson3d(10, 9, 8), (10, 9, 8), 32, 1e-4, True),
    "nonsym": (lambda: random_nonsym_dd(np.random.default_rng(12), 20, 16), (20, 16, 1), 10, 1e-3, False),
    "p2d_exact": (lambda: poisson2d(16, 12), (16, 12, 1), 8, 0.0, True),
}

FORCED = [
    ("pivot_in_memory", dict(pivot_lds_max=0), ["p3d", "nonsym", "p2d_exact"]),
    ("trinv_12_blocks", dict(pivot_lds_max=0, trinv8_max=0), ["p3d", "nonsym"]),
    ("trinv_per_wave", dict(pivot_lds_max=0, trinv8_max=0, trinv12_max=0), ["p3d", "nonsym", "p2d_exact"]),
    ("complement_two_slots", dict(qr_reg1_max=0), ["p3d", "nonsym"]),
    ("complement_in_memory", dict(qr_reg1_max=0, qr_reg2_max=0), ["p3d", "nonsym"]),
    ("complement_q_without_wy", dict(wy_max=0), ["p3d", "nonsym"]),
    ("gram_partners_shared", dict(gram_splits_max=2), ["p3d", "nonsym"]),
    ("gram_single_partial", dict(gram_splits_max=1), ["p3d"]),
    ("schur_no_pointer_table", dict(schur_ptab_max=0), ["p3d", "nonsym", "p2d_exact"]),
    ("schur_offsets_in_memory", dict(schur_noff_max=0, schur_ptab_max=3), ["p3d", "nonsym"]),
    ("basis_by_householder", dict(cholqr=0), ["p3d", "nonsym"]),
    # every level crowded: four Gram partials per cluster, the complement's
    # columns wave by wave, U by Householder QR (the settings of the batched
    # workload's large levels)
    ("crowded_settings", dict(crowded_min=0), ["p3d", "nonsym", "p2d_exact"]),
    ("dense_panels_16", dict(dense_panel=16), ["p3d", "p2d_exact"]),
    # forward solve step in one launch / in two
    ("apply_one_launch", dict(apply_fwd=1), ["p3d", "nonsym", "p2d_exact"]),
    ("apply_two_launches", dict(apply_fwd=2), ["p3d", "nonsym", "p2d_exact"]),
    # rank revelation by the pivoted Householder QR of F^T at eps >= 1e-5 (its
    # own kernel, k_qrcp; compared at the pivoted-QR bar, 1e-9 here)
    ("rank_by_pivoted_qr", dict(compression=1), ["p3d", "nonsym"]),
    ("rank_by_pivoted_qr_in_memory", dict(compression=1, pivot_lds_max=0), ["p3d", "nonsym"]),
]

FORCED_CASES = [(v, kn, inp) for v, kn, inputs in FORCED for inp in inputs]


@pytest.mark.parametrize("variant,kn,inp", FORCED_CASES, ids=[f"{v}-{i}" for v, _, i in FORCED_CASES])
def test_forced_variant(P, variant, kn, inp):
    mk, dims, leaf, eps, sym = SMALL[inp]
    A = mk()
    print(f"[variants] {variant} on {inp}: {kn}", flush=True)
    with knobs(P, **kn):
        fo, F, st = compare_factor(P, A, dims, leaf, eps, sym)
    _check_solve(P, fo, F, A)


@pytest.mark.parametrize("name,mk,dims,leaf,sym", [
    ("p2d_leaf144", lambda: poisson2d(48, 48), (48, 48, 1), 144, True),
    ("convdiff_leaf144", lambda: convdiff2d_upwind(48, 50.0, 0.3), (48, 48, 1), 144, False),
])
def test_pivoted_qr_large_clusters(P, name, mk, dims, leaf, sym):
    """The pivoted-QR route on clusters of 144 (memory-resident pivot kernel)
    at eps = 1e-7: ranks bit-exact, solves to 1e-8, factor entries to 1e-6
    wherever the input determines them (on the 2D Poisson input one cluster's
    pivots are decided by rounding: the oracle's own coarse basis of it moves
    by 0.35 under a 1e-15 perturbation of A)."""
    A = mk()
    print(f"[variants] pivoted QR {name}", flush=True)
    fo, F, st = compare_factor(P, A, dims, leaf, 1e-7, sym, stable_only=True)
    assert st["levels_compared"] >= 1
    assert st["max_lowrank_m"] == 144
    _check_solve(P, fo, F, A)


@pytest.mark.parametrize("factor_of_floor", [0.5, 2.0])
def test_noise_floor_decision(P, factor_of_floor):
    """Reading R12 on the device: fill at half the 1e-12 ||A_ss||_F floor is
    dropped (k = 0), at twice the floor it is compressed; ranks, factor and
    solve as the oracle's."""
    d0 = 1e-6
    _, leaf = scaled_coupling_poisson(1.0)
    r1 = fill_ratio_of_c1(scaled_coupling_poisson(d0)[0], leaf) / d0
    A, _ = scaled_coupling_poisson(factor_of_floor * 1e-12 / r1)
    print(f"[variants] noise floor x{factor_of_floor}", flush=True)
    fo, F, st = compare_factor(P, A, (4, 4, 1), 4, 1e-6, True)
    assert (F.ranks(0)[1] == 0) == (factor_of_floor < 1.0)
    _check_solve(P, fo, F, A)


@pytest.mark.parametrize("wave", [None, 1], ids=["default", "waves_everywhere"])
@pytest.mark.parametrize("case", ["p3d_mixed", "convdiff_fp64"])
def test_solve_columns_independent_bitwise(P, case, wave):
    """Each column of a solve with several right-hand sides equals that
    column solved alone, bit for bit: every sweep takes a column's sums in an
    order that does not depend on how many columns share the launch (the
    forward step in one launch or two, the own products one wave per cluster
    or in 64-row chunks, four or eight columns per backward pass)."""
    if case == "p3d_mixed":
        A, dims, eps, sym, prec = poisson3d(14, 14, 14), (14, 14, 14), 1e-4, 1, P.HS_MIXED
    else:
        A, dims, eps, sym, prec = convdiff2d_upwind(96, 40.0, 0.7), (96, 96, 1), 1e-3, 0, P.HS_FP64
    settings = {} if wave is None else {"apply_wave": wave}
    with knobs(P, **settings):
        F = P.Factor(A.row_ptr, A.col_idx, A.val, dims, eps, 64, symmetric=sym, precision=prec)
        B = torch.tensor(np.random.default_rng(21).uniform(-1, 1, (8, A.n)), device="cuda")
        X8 = F.solve(B).cpu().numpy()
        X5 = F.solve(B[:5].contiguous()).cpu().numpy()
        for j in range(8):
            xj = F.solve(B[j:j + 1].contiguous()).cpu().numpy()
            assert np.array_equal(xj[0], X8[j]), j
            if j < 5:
                assert np.array_equal(xj[0], X5[j]), j
        F.free()
    print(f"[variants] columns independent: {case} {settings}", flush=True)


@pytest.mark.parametrize("case", ["p3d_big_clusters", "convdiff_mixed", "batch_mixed"])
def test_apply_wave_form_bitwise(P, case):
    """One right-hand side: the own products one wave per cluster (clusters
    up to 128 unknowns) and in 64-row workgroup chunks take the same sums in
    the same order, so the solves agree bit for bit; float32 and float64
    levels, colours above 128 unknowns falling back to the chunked form."""

    rng = np.random.default_rng(11)
    if case == "p3d_big_clusters":
        A = poisson3d(12, 12, 12)
        mk = lambda: P.Factor(A.row_ptr, A.col_idx, A.val, (12, 12, 12), 1e-4, 200, symmetric=1)  # noqa: E731
        n = A.n
    elif case == "convdiff_mixed":
        A = convdiff2d_upwind(96, 40.0, 0.7)
        mk = lambda: P.Factor(A.row_ptr, A.col_idx, A.val, (96, 96, 1), 1e-3, 64, symmetric=0,  # noqa: E731
                              precision=P.HS_MIXED, coarse_fp64_dofs=1000)
        n = A.n
    else:
        As = [convdiff2d_upwind(s, pe, th) for s, pe, th in ((64, 10.0, 0.3), (80, 60.0, 2.0), (48, 90.0, 4.0))]
        systems = [(a.row_ptr, a.col_idx, a.val, (int(round(a.n ** 0.5)),) * 2 + (1,)) for a in As]
        mk = lambda: P.Factor.batch(systems, 1e-3, 64, symmetric=0, precision=P.HS_MIXED)  # noqa: E731
        n = sum(a.n for a in As)
    b = torch.tensor(rng.uniform(-1, 1, (1, n)), device="cuda")
    xs = []
    for mode in (0, 1):
        with knobs(P, apply_wave=mode):
            F = mk()
        xs.append(F.solve(b).cpu().numpy())
        F.free()
    print(f"[variants] apply_wave {case}: n={n}", flush=True)
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("nrhs", [1, 5])
def test_apply_launch_forms_bitwise(P, nrhs):
    """The forward step in one launch (neighbour workgroups form z_s[:f]
    again) and in two (z_s once), and the own products cut into 64-row
    chunks: the same sums in the same order, so the solves agree bit for bit
    (clusters up to 324 unknowns, several chunks each)."""
    A = poisson3d(12, 12, 12)
    b = torch.tensor(np.random.default_rng(9).uniform(-1, 1, (nrhs, A.n)), device="cuda")
    xs = []
    for mode in (0, 1, 2):
        with knobs(P, apply_fwd=mode):
            F = P.Factor(A.row_ptr, A.col_idx, A.val, (12, 12, 12), 1e-4, 200, symmetric=1)
        xs.append(F.solve(b).cpu().numpy())
        F.free()
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
