"""Autotuner of the kernel-variant thresholds (hs_config_set).

The thresholds pick between kernel variants that compute the same numbers up
to rounding and differ in where their working data lives and how work is
split: the forward solve step in one launch or two (apply_fwd), the own
products of a one-right-hand-side solve one wave per cluster (apply_wave), the panel
width of the dense levels (dense_panel), how many fill partners share a Gram
workgroup (gram_splits_max), how large a cluster may keep its working matrix
in LDS (pivot_lds_max), whether the complement's columns go through the
compact WY form (wy_max) and the basis U through Cholesky QR (cholqr), and
the same three on crowded levels (gram_splits_crowded, wy_max_crowded,
cholqr_crowded, with crowded_min clusters per colour).  ``autotune`` times a representative workload (one
factorization and one Krylov solve, on the caller's matrices) under each
candidate setting, one parameter at a time from the current values, keeps a
change only when it is faster by more than ``min_gain`` and the solution
agrees with the reference setting's to ``tol``, and leaves the best setting
installed (process-wide) for the factorizations that follow.
"""

from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib as L

# parameter -> candidate values (the defaults are among them)
CANDIDATES: Dict[str, List[float]] = {
    "apply_fwd": [0, 1, 2],
    "apply_wave": [0, 256, 1024, 4096],
    "apply_split_nrhs_max": [1, 64],
    "dense_panel": [64, 128],
    "gram_splits_max": [64, 128, 256],
    "gram_splits_crowded": [2, 4, 8, 256],
    "crowded_min": [128, 512, 2048],
    "pivot_lds_max": [64, 128],
    "wy_max": [0, 128],
    "cholqr": [0, 1],
    "wy_max_crowded": [0, 128],
    "cholqr_crowded": [0, 1],
}


def _run(systems, eps, leaf, symmetric, precision, B, krylov, tol, maxit):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = L.Factor.batch(systems, eps, leaf, symmetric=symmetric, precision=precision)
    if krylov == "cg":
        X, it, rel, ok = F.pcg(B, tol, maxit)
    elif krylov == "gmres":
        X, it, rel, ok = F.gmres(B, tol, maxit, 30)
    else:
        X, it, rel, ok = F.solve(B), 0, np.zeros(1), True
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    F.free()
    return dt, X, int(it), bool(ok)


def autotune(systems: Sequence[Tuple], eps: float, leaf: int = 64, symmetric: int = -1,
             precision: int = L.HS_FP64, B=None, krylov: str = "gmres", krylov_tol: float = 1e-10,
             maxit: int = 300, repeats: int = 2, min_gain: float = 0.03, tol: float = 1e-8,
             candidates: Optional[Dict[str, List[float]]] = None, log=None) -> Dict[str, float]:
    """Tune the thresholds on ``systems`` = [(row_ptr, col_idx, val, dims), ...]
    (a batch as for Factor.batch; device or host CSR).  B: right-hand sides
    as a (nrhs, n) CUDA float64 tensor (default: ones).  krylov: "gmres",
    "cg" or "solve" (one application).  Returns the chosen values of every
    tuned parameter; they stay installed (config_reset() restores the
    defaults)."""
    import torch

    cands = CANDIDATES if candidates is None else candidates
    if B is None:
        n = 0
        for rp, _, _, _ in systems:
            n += int(rp.shape[0]) - 1 if hasattr(rp, "shape") else len(rp) - 1
        B = torch.ones((1, n), dtype=torch.float64, device="cuda")

    def timed():
        best = None
        X = None
        for _ in range(max(1, repeats)):
            dt, X, it, ok = _run(systems, eps, leaf, symmetric, precision, B, krylov, krylov_tol, maxit)
            best = dt if best is None else min(best, dt)
        return best, X, ok

    _run(systems, eps, leaf, symmetric, precision, B, krylov, krylov_tol, maxit)  # warm-up
    t_best, X_ref, ok_ref = timed()
    if log:
        log(f"autotune: current setting {t_best * 1e3:.1f} ms")
    chosen = {}
    for name, values in cands.items():
        cur = L.config_get(name)
        chosen[name] = cur
        for v in values:
            if v == cur:
                continue
            L.config_set(name, v)
            dt, X, ok = timed()
            err = float(torch.linalg.norm(X - X_ref) / torch.linalg.norm(X_ref))
            good = ok == ok_ref and err <= tol and dt < t_best * (1.0 - min_gain)
            if log:
                log(f"autotune: {name}={v:g}: {dt * 1e3:.1f} ms, solution differs by {err:.1e}"
                    f"{' (kept)' if good else ''}")
            if good:
                t_best, chosen[name] = dt, v
            L.config_set(name, chosen[name])
    return chosen
