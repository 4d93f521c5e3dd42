"""Precision study (test infrastructure, CPU only): how the preconditioner
degrades when the per-cluster dense algebra of Sec. 2.1 (the LU of A_ss and
F_ff, the triangular solves, the complement's Householder QR, the Schur
products of Eq. elim) runs in float32 instead of float64 on every level but
the two coarsest, compared with float32 storage of blocks and records only.

Each setting factors with the oracle and runs its right-preconditioned
GMRES(30) to 1e-10; the float32 arithmetic is emulated by evaluating the
oracle's dense helpers on float32 copies of their operands (numpy / LAPACK
float32 routines) and widening the results.  Settings:

  fp64      the oracle as it is
  storage   float64 arithmetic, every block and record rounded to float32
            after the level that produced it (the library's mixed form)
  fp32      float32 arithmetic and storage on the fine levels; the rank
            revelation (Eq. lra) stays float64
  fp32rank  as fp32, and the rank revelation in float32 as well

Usage: python -m oracle.precision_study [--quick]
"""

from __future__ import annotations

import argparse
import contextlib
import time

import numpy as np

from . import hs_oracle as H

_F32 = {"on": False, "rank": False, "store": False}


def _f32(x):
    return np.asarray(x, dtype=np.float32)


def _wrap(fn, rank=False):
    def g(*args, **kw):
        if _F32["on"] and (not rank or _F32["rank"]):
            args = [(_f32(a) if isinstance(a, np.ndarray) else a) for a in args]
            out = fn(*args, **kw)
            def widen(o):
                return o.astype(np.float64) if isinstance(o, np.ndarray) and o.dtype.kind == "f" else o

            return tuple(widen(o) for o in out) if isinstance(out, tuple) else widen(out)
        return fn(*args, **kw)

    return g


def _lu32(a):
    """Doolittle LU without pivoting in float32 (reading R9's algorithm)."""
    if not _F32["on"]:
        return _ORIG["lu_nopiv"](a)
    n = a.shape[0]
    lu = np.array(a, dtype=np.float32, copy=True)
    for j in range(n):
        p = lu[j, j]
        if p == 0.0 or not np.isfinite(p):
            raise H.Breakdown(f"pivot {j} of a {n}x{n} block is {p}")
        lu[j + 1 :, j] /= p
        lu[j + 1 :, j + 1 :] -= np.outer(lu[j + 1 :, j], lu[j, j + 1 :])
    return (np.tril(lu, -1) + np.eye(n, dtype=np.float32)).astype(np.float64), np.triu(lu).astype(np.float64)


def _schur32(blocks, nb, nsz, EL, ER):
    """Eq. elim with the products in float32 (arithmetic) and the updated
    blocks rounded to float32 (storage)."""
    if _F32["on"]:
        EL, ER = _f32(EL), _f32(ER)
    _ORIG["_schur"](blocks, nb, nsz, EL, ER)
    if _F32["store"]:
        for a in nb:
            for b in nb:
                blocks[(a, b)] = blocks[(a, b)].astype(np.float32).astype(np.float64)


_ORIG = {}
_PATCH = {
    "lu_nopiv": lambda: _lu32,
    "_lsolve": lambda: _wrap(_ORIG["_lsolve"]),
    "_usolve": lambda: _wrap(_ORIG["_usolve"]),
    "_lu_solve": lambda: _wrap(_ORIG["_lu_solve"]),
    "_lu_solve_t": lambda: _wrap(_ORIG["_lu_solve_t"]),
    "_right_usolve": lambda: _wrap(_ORIG["_right_usolve"]),
    "householder_complement": lambda: _wrap(_ORIG["householder_complement"]),
    "qrcp_truncated": lambda: _wrap(_ORIG["qrcp_truncated"], rank=True),
    "_schur": lambda: _schur32,
}


@contextlib.contextmanager
def _patched():
    for name in _PATCH:
        _ORIG[name] = getattr(H, name)
    try:
        for name, mk in _PATCH.items():
            setattr(H, name, mk())
        yield
    finally:
        for name, fn in _ORIG.items():
            setattr(H, name, fn)


def _round_level(level):
    """Round a finished level's records to float32 (storage)."""
    for r in level.records:
        if r is None:
            continue
        for name in ("L", "Uu", "Lf", "Uf", "U", "VL", "VR", "ER", "EL"):
            v = getattr(r, name, None)
            if isinstance(v, np.ndarray):
                setattr(r, name, v.astype(np.float32).astype(np.float64))


def run_setting(A, dims, leaf, eps, symmetric, setting, b):
    nlev = len(H.symbolic_analysis(A.row_ptr, A.col_idx, dims, leaf)[1])
    fine = lambda lvl: lvl < nlev - 2  # noqa: E731
    _F32["on"] = setting in ("fp32", "fp32rank") and fine(0)
    _F32["rank"] = setting == "fp32rank"
    _F32["store"] = setting != "fp64" and fine(0)

    def progress(lvl, level):
        if setting != "fp64" and fine(lvl):
            _round_level(level)
        _F32["on"] = setting in ("fp32", "fp32rank") and fine(lvl + 1)
        _F32["store"] = setting != "fp64" and fine(lvl + 1)

    t0 = time.perf_counter()
    with _patched():
        try:
            fo = H.factor(A.row_ptr, A.col_idx, A.val, dims, leaf, eps, symmetric, progress=progress)
        except H.Breakdown as e:
            return {"setting": setting, "breakdown": str(e)}
        finally:
            _F32["on"] = _F32["store"] = False
    tf = time.perf_counter() - t0
    x, it, rel = H.gmres(A.row_ptr, A.col_idx, A.val, b, lambda R: H.solve(fo, R), 1e-10, 300)
    return {"setting": setting, "gmres_iterations": int(it), "relres": float(rel), "factor_s": round(tf, 1)}


def main():
    from workloads import convdiff2d_upwind, poisson3d

    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    cases = [("convdiff 128^2 Pe 50", convdiff2d_upwind(128, 50.0, 0.3), (128, 128, 1), False),
             ("poisson 24^3", poisson3d(24, 24, 24), (24, 24, 24), True)]
    if not args.quick:
        cases.insert(1, ("convdiff 256^2 Pe 90", convdiff2d_upwind(256, 90.0, 1.1), (256, 256, 1), False))
    for name, A, dims, sym in cases:
        b = np.random.default_rng(0).uniform(-1, 1, A.n)
        for eps in (1e-3,):
            for setting in ("fp64", "storage", "fp32", "fp32rank"):
                r = run_setting(A, dims, 64, eps, sym, setting, b)
                print(f"{name:22s} eps {eps:g} {setting:9s} {r}", flush=True)


if __name__ == "__main__":
    main()
