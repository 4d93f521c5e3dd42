"""Benchmark: unknowns/s to factor and solve to relative residual 1e-10, the
mixed-precision form against the float64 form.

Workload (default): 3D 7-point Poisson on a 64^3 grid (N = 262,144), FP64 CSR,
leaves of 64 unknowns, eps = 1e-4, the factorization used as CG
preconditioner for 8 right-hand sides uniform on [-1, 1), stopping at
relative residual 1e-10 for every column.  One step = hs_factor + hs_pcg
(symbolic analysis, numeric factorization and the preconditioned solve of all
8 right-hand sides) + hs_free, with the CSR and the right-hand sides already
resident in HBM.  value = N * steps / seconds of the mixed form (float32
blocks and records, Schur products on the bfloat16 units, float64 coarse
levels and Krylov vectors); the float64 form is timed the same way and
reported beside it.

Also reported: the Schur-complement kernel against the HBM roofline (its
algorithmic bytes per launch over its average launch time, HIP events on the
library's stream inside the timed region) and the CPU oracle timed on a
bounded sample of the same workload family on the host cores.

Batched workload (--workload batch): 256 independent 2D upwind
convection-diffusion systems (sides uniform in [64, 512], Peclet uniform in
[1, 100], random direction; about 2.7e7 unknowns), one right-hand side each,
GMRES(30) to 1e-10 per system.  Systems are factored together with
hs_factor_batch in groups whose measured device footprint fits the memory
budget; one step = every group's hs_factor_batch + hs_gmres + hs_free.

Serving workload (--workload serve): a Poisson stream of solve requests
(60 % 3D lognormal diffusion with sides 32..96, 40 % 2D convection-diffusion
with sides 256..1024, 1-16 right-hand sides, 30 % operator reuse) served by
the library's request loop at rho times its capacity measured on a burst;
value = unknowns x right-hand sides solved per second, with p50 / p99
latency.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--side 64] [--forms both|mixed|fp64]
                       [--workload poisson64|batch|serve] [--batch-count 256] [--budget-gb 200]
                       [--requests 100] [--rho 0.8] [--cap-gb 200] [--workers 2]
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_schur_hbm_traffic_poisson64.md")


def schur_source_digest() -> str:
    """Digest of the Schur-update kernel's source (its section of k_factor.hip
    and the MFMA tile core it is built on)."""
    csrc = os.path.join(ROOT, "paper_1712_07297_amd", "csrc")

    def section(name, a, b):
        with open(os.path.join(csrc, name)) as fh:
            text = fh.read()
        i = text.index(a)
        return text[i : text.index(b, i)]

    h = hashlib.sha256()
    h.update(section("k_factor.hip", "// " + "=" * 60 + " Schur update", "// " + "=" * 64 + " assembly").encode())
    h.update(section("device_common.h", "// " + "-" * 60 + " MFMA tile core", "// " + "-" * 60 + " cooperative GEMM").encode())
    return h.hexdigest()[:16]


def measured_traffic(element: str):
    """HBM bytes per k_schur<element> launch from the committed FETCH_SIZE /
    WRITE_SIZE passes on this workload, or None when the kernel changed since."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("traffic_bytes_per_launch_", "kernel_source_digest:")))
    if vals.get("kernel_source_digest", "").strip() != schur_source_digest():
        return None
    v = vals.get(f"traffic_bytes_per_launch_{element}")
    return float(v) if v is not None else None


def cpu_baseline(side: int = 24):
    """The oracle (plain numpy FP64) on a side^3 Poisson sample of the same
    workload family: factor + PCG for 8 RHS to 1e-10."""
    import oracle as O
    from workloads import config2

    try:
        from threadpoolctl import threadpool_info

        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    p = config2(side=side, nrhs=8)
    t0 = time.perf_counter()
    fo = O.factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.leaf, p.eps, True)
    X, it, rel = O.pcg(p.A.row_ptr, p.A.col_idx, p.A.val, p.B, lambda R: O.solve(fo, R), p.tol, 200)
    dt = time.perf_counter() - t0
    assert rel.max() <= p.tol
    return {
        "value": p.A.n / dt,
        "unit": "unknowns/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"3D Poisson {side}^3 (N={p.A.n}), leaf 64, eps 1e-4, 8 RHS, PCG to 1e-10: one factor+solve in {dt:.1f} s",
    }


def run_form(P, torch, p, rp, ci, va, B, X, precision, steps, warmup, n, profile=False):
    """Warm-up, then `steps` timed steps of one precision form; returns its
    record (time, convergence, Schur roofline)."""

    split = {"factor": 0.0, "solve": 0.0}

    def step():
        t0 = time.perf_counter()
        F = P.Factor(rp, ci, va, p.dims, p.eps, p.leaf, symmetric=1, precision=precision)
        t1 = time.perf_counter()
        _, it, rel, ok = F.pcg(B, p.tol, 200, X=X)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        split["factor"] += t1 - t0
        split["solve"] += t2 - t1
        info = F.info()
        F.free()
        return it, rel, ok, info

    name = "mixed" if precision == P.HS_MIXED else "fp64"
    for w in range(warmup):
        step()
        print(f"{name}: warmup step {w + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    P.profile_reset()
    # the dominant kernel is timed by events around its launches; the rest
    # runs as in production unless every family is profiled
    P.profile_select("" if profile else ("schur_f32" if precision == P.HS_MIXED else "schur"))
    P.profile_enable(True)
    torch.cuda.synchronize()
    split["factor"] = split["solve"] = 0.0
    t0 = time.perf_counter()
    its, rels, oks = [], [], []
    info = None
    for k in range(steps):
        it, rel, ok, info = step()
        print(f"{name}: timed step {k + 1}/{steps} done", file=sys.stderr, flush=True)
        its.append(it)
        rels.append(float(rel.max()))
        oks.append(ok)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    P.profile_enable(False)
    if profile:
        fams = ["gram", "pivot", "fill", "nbr", "schur", "schur_f32", "merge", "apply", "spmv", "dense",
                "host_symbolic", "host_plan", "host_upload", "host_alloc", "host_sync", "host_solve_plan"]
        prof = {f: round(P.profile_read(f)["seconds"] / steps, 4) for f in fams}
        print(f"{name}: seconds per step by family {json.dumps(prof)}", file=sys.stderr, flush=True)
    # dominant kernel: the Schur updates of the levels stored in the form's
    # bulk precision (float32 levels in the mixed form, all levels in FP64)
    schur = P.profile_read("schur_f32" if precision == P.HS_MIXED else "schur")
    # independent check of the final residual (device SpMV by torch, FP64)
    A_t = torch.sparse_csr_tensor(rp, ci.to(torch.int64), va, size=(n, n))
    R = B.T - (A_t @ X.T)
    relres = (torch.linalg.norm(R, dim=0) / torch.linalg.norm(B.T, dim=0)).max().item()
    rec = {
        "value": n * steps / dt,
        "ms_per_step": dt / steps * 1e3,
        "factor_ms": split["factor"] / steps * 1e3,
        "solve_ms": split["solve"] / steps * 1e3,
        "pcg_iterations": its,
        "relres_max": max(rels),
        "relres_check": relres,
        "converged": all(oks) and relres <= p.tol * 1.01,
        "levels": info.nlevels,
        "colour_batches": info.ncolors_total,
        "factor_gflop": info.factor_flops / 1e9,
        "factor_bytes_records": info.factor_bytes,
    }
    if schur["launches"] > 0 and schur["seconds"] > 0:
        achieved = schur["bytes"] / schur["seconds"] / 1e9
        rec["roofline"] = {
            "kernel": f"k_schur<{'float' if precision == P.HS_MIXED else 'double'}> (Schur-complement update, Eq. elim)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "launches": schur["launches"],
            "avg_launch_ms": schur["seconds"] / schur["launches"] * 1e3,
            "algorithmic_bytes_per_launch": schur["bytes"] / schur["launches"],
            "achieved_tflops": schur["flops"] / schur["seconds"] / 1e12,
        }
    return rec


def run_batch(args):
    """The batched convection-diffusion workload, mixed and float64 forms."""
    import torch

    import paper_1712_07297_amd as P
    from workloads import config4_batch

    dev = torch.device("cuda:0")
    probs = config4_batch(count=args.batch_count)
    ns = [p.A.n for p in probs]
    ntot = int(sum(ns))
    sys_dev = [(torch.tensor(p.A.row_ptr, device=dev), torch.tensor(p.A.col_idx, device=dev),
                torch.tensor(p.A.val, device=dev), p.dims) for p in probs]
    rhs = [torch.tensor(np.ascontiguousarray(p.B[:, 0]), device=dev) for p in probs]
    torch.cuda.synchronize()
    budget = args.budget_gb * 1e9

    def run_group(idx, precision):
        F = P.Factor.batch([sys_dev[i] for i in idx], 1e-3, 64, symmetric=0, precision=precision)
        B = torch.cat([rhs[i] for i in idx]).reshape(1, -1)
        _, it, rel, ok = F.gmres(B, 1e-10, 300, 30)
        info = F.info()
        F.free()
        return it, float(np.max(rel)), ok, info

    out_forms = {}
    forms = {"both": [P.HS_MIXED, P.HS_FP64], "mixed": [P.HS_MIXED], "fp64": [P.HS_FP64]}[args.forms]
    for prec in forms:
        name = "mixed" if prec == P.HS_MIXED else "fp64"
        # footprint per unknown from a calibration group (also the warm-up)
        cal = list(range(min(8, len(probs))))
        _, _, _, info = run_group(cal, prec)
        per_unknown = info.peak_device_bytes / sum(ns[i] for i in cal)
        cap = max(1, int(budget / (1.25 * per_unknown)))
        groups, cur, acc = [], [], 0
        for i in range(len(probs)):
            if cur and acc + ns[i] > cap:
                groups.append(cur)
                cur, acc = [], 0
            cur.append(i)
            acc += ns[i]
        groups.append(cur)
        print(f"batch {name}: {len(groups)} group(s), {per_unknown:.0f} B/unknown", file=sys.stderr, flush=True)
        times, its, rels, oks, peaks = [], [], [], [], []
        if args.profile:
            P.profile_reset()
            P.profile_enable(True)
        for st in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for g in groups:
                it, rel, ok, info = run_group(g, prec)
                its.append(it)
                rels.append(rel)
                oks.append(ok)
                peaks.append(info.peak_device_bytes)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            print(f"batch {name}: step {st + 1}/{args.steps} {times[-1]:.2f} s", file=sys.stderr, flush=True)
        if args.profile:
            P.profile_enable(False)
            fams = ["gram", "pivot", "fill", "nbr", "schur", "schur_f32", "merge", "apply", "spmv", "dense",
                    "host_symbolic", "host_plan", "host_upload", "host_alloc", "host_sync",
                    "host_solve_plan"]
            prof = {f: round(P.profile_read(f)["seconds"] / args.steps, 4) for f in fams}
            print(f"batch {name}: seconds per step by family {json.dumps(prof)}", file=sys.stderr, flush=True)
        dt = float(np.median(times))
        out_forms[name] = {
            "value": ntot / dt,
            "ms_per_step": dt * 1e3,
            "groups": len(groups),
            "gmres_iterations_max": int(max(its)),
            "relres_max": float(max(rels)),
            "converged": bool(all(oks)) and max(rels) <= 1e-10,
            "peak_device_gb": float(max(peaks)) / 1e9,
        }
    head_name = "mixed" if "mixed" in out_forms else "fp64"
    head = out_forms[head_name]
    out = {
        "metric": "unknowns/s factor+solve to 1e-10 residual (mixed vs FP64)",
        "value": head["value"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage + bf16x3 MFMA Schur, f64 Krylov" if head_name == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"batch of {len(probs)} 2D upwind convection-diffusion systems (sides 64..512, N total {ntot}), "
                        "leaf 64, eps 1e-3, hs_factor_batch + GMRES(30) to 1e-10 per system, 1 RHS each",
            "form": head_name,
            **{k: v for k, v in head.items() if k not in ("value", "ms_per_step")},
        },
    }
    if "fp64" in out_forms and head_name != "fp64":
        out["fp64"] = out_forms["fp64"]
        out["mixed_over_fp64"] = head["value"] / out_forms["fp64"]["value"]
    print(json.dumps(out))


def run_serve(args):
    """The serving stream: Poisson arrivals of solve requests (60 % 3D
    lognormal diffusion, CG; 40 % 2D convection-diffusion, GMRES(30); 1-16
    right-hand sides; 30 % reuse an earlier operator), mixed form, served by
    the library's request loop at a load of rho times its measured capacity."""
    import torch

    import paper_1712_07297_amd as P
    from workloads import build_request_operator, serving_stream

    dev = torch.device("cuda:0")
    reqs = serving_stream(args.seed, args.requests, rate=1.0)
    ops, rhs = {}, []
    rng = np.random.default_rng(args.seed + 1)
    t0 = time.perf_counter()
    for r in reqs:
        if r.op_key not in ops:
            A, dims, _, sym = build_request_operator(r)
            ops[r.op_key] = (torch.tensor(A.row_ptr, device=dev), torch.tensor(A.col_idx, device=dev),
                             torch.tensor(A.val, device=dev), dims, int(sym), A.n)
        n = ops[r.op_key][5]
        rhs.append(torch.tensor(rng.uniform(-1.0, 1.0, (r.nrhs, n)), device=dev))
    torch.cuda.synchronize()
    print(f"serve: {len(ops)} operators, {len(reqs)} requests prepared in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)

    def make_server():
        return P.Server(hbm_cap_gb=args.cap_gb, workers=args.workers, max_batch=32, max_new_ops=8)

    def submit(srv, i, key_base=0):
        r = reqs[i]
        rp, ci, va, dims, sym, n = ops[r.op_key]
        return srv.submit(key_base + r.op_key, rp, ci, va, dims, rhs[i], eps=1e-3, leaf=64, symmetric=sym,
                          precision=P.HS_MIXED, tol=1e-10, maxit=300)

    # capacity: a burst of the first requests on a separate server (warm-up too)
    cal = min(args.calibrate, len(reqs))
    srv = make_server()
    tc = time.perf_counter()
    ts = [submit(srv, i) for i in range(cal)]
    for t in ts:
        srv.wait(t)
    mu = cal / (time.perf_counter() - tc)
    srv.close()
    lam = args.rho * mu
    print(f"serve: capacity {mu:.2f} requests/s from a burst of {cal}; arrival rate {lam:.2f}/s", file=sys.stderr,
          flush=True)

    srv = make_server()
    arrivals = np.array([r.t_arrival for r in reqs]) / lam  # unit-rate stream scaled to lam
    tickets = []
    torch.cuda.synchronize()
    start = time.perf_counter()
    for i in range(len(reqs)):
        delay = start + arrivals[i] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(submit(srv, i))
        if (i + 1) % 25 == 0:
            print(f"serve: {i + 1}/{len(reqs)} submitted", file=sys.stderr, flush=True)
    results = [srv.wait(t)[1] for t in tickets]
    wall = time.perf_counter() - start
    st = srv.stats()
    srv.close()
    ok = all(r["status"] == 0 for r in results) and max(r["relres"] for r in results) <= 1e-10
    out = {
        "metric": "unknowns/s factor+solve to 1e-10 residual; p50/p99 latency (serving)",
        "value": st["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage + bf16x3 MFMA Schur, f64 Krylov",
        "data": "synthetic",
        "config": {
            "workload": f"serving stream of {len(reqs)} requests ({len(ops)} operators): 60% 3D lognormal diffusion "
                        "(sides 32..96, CG), 40% 2D convection-diffusion (sides 256..1024, GMRES(30)), 1-16 RHS, "
                        "30% operator reuse, Poisson arrivals, eps 1e-3, tol 1e-10",
            "rho": args.rho,
            "arrival_rate_per_s": lam,
            "capacity_per_s": mu,
            "p50_latency_s": st["p50_latency_s"],
            "p99_latency_s": st["p99_latency_s"],
            "mean_queue_s": st["mean_queue_s"],
            "requests_per_s": st["requests_per_s"],
            "completed": st["completed"],
            "reused": st["reused"],
            "batches": st["batches"],
            "factored_ops": st["factored_ops"],
            "evictions": st["evictions"],
            "peak_held_gb": st["peak_held_bytes"] / 1e9,
            "cap_gb": args.cap_gb,
            "workers": args.workers,
            "max_relres": max(r["relres"] for r in results),
            "converged": ok,
        },
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side", type=int, default=64)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--forms", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=24)
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--workload", choices=["poisson64", "batch", "serve"], default="poisson64")
    ap.add_argument("--requests", type=int, default=100, help="serve workload: requests in the stream")
    ap.add_argument("--rho", type=float, default=0.8, help="serve workload: load over measured capacity")
    ap.add_argument("--cap-gb", type=float, default=200.0, help="serve workload: device memory cap")
    ap.add_argument("--workers", type=int, default=2, help="serve workload: batches in flight")
    ap.add_argument("--calibrate", type=int, default=12, help="serve workload: burst size for the capacity")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--budget-gb", type=float, default=200.0, help="device memory per batched group")
    ap.add_argument("--profile", action="store_true", help="per-family times (HIP events, host wall) to stderr")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return

    import torch

    import paper_1712_07297_amd as P
    from workloads import config2

    dev = torch.device("cuda:0")
    p = config2(side=args.side, nrhs=args.nrhs)
    n = p.A.n
    rp = torch.tensor(p.A.row_ptr, device=dev)
    ci = torch.tensor(p.A.col_idx, device=dev)
    va = torch.tensor(p.A.val, device=dev)
    B = torch.tensor(np.ascontiguousarray(p.B.T), device=dev)  # (nrhs, n) = column-major n x nrhs
    X = torch.empty_like(B)
    torch.cuda.synchronize()

    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024 // 8, dtype=torch.float64, device=dev)  # 64 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    forms = {"both": [P.HS_MIXED, P.HS_FP64], "mixed": [P.HS_MIXED], "fp64": [P.HS_FP64]}[args.forms]
    recs = {}
    for prec in forms:
        recs["mixed" if prec == P.HS_MIXED else "fp64"] = run_form(P, torch, p, rp, ci, va, B, X, prec, args.steps,
                                                                   args.warmup, n, args.profile)
    head = recs.get("mixed", recs.get("fp64"))
    head_name = "mixed" if "mixed" in recs else "fp64"
    out = {
        "metric": "unknowns/s factor+solve to 1e-10 residual (mixed vs FP64)",
        "value": head["value"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage + bf16x3 MFMA Schur, f64 Krylov" if head_name == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D 7-point Poisson {args.side}^3 (N={n}), leaf 64, eps 1e-4, PCG preconditioner, {args.nrhs} RHS to relative residual 1e-10",
            "form": head_name,
            "factor_ms": head["factor_ms"],
            "solve_ms": head["solve_ms"],
            "pcg_iterations": head["pcg_iterations"],
            "relres_max": head["relres_max"],
            "relres_check": head["relres_check"],
            "converged": head["converged"],
            "levels": head["levels"],
            "colour_batches": head["colour_batches"],
            "factor_gflop": head["factor_gflop"],
            "factor_bytes_records": head["factor_bytes_records"],
        },
    }
    if args.side == 64 and args.nrhs == 8:
        for name, rec in recs.items():
            if "roofline" in rec:
                rec["roofline"]["traffic"] = measured_traffic("float" if name == "mixed" else "double")
    if "roofline" in head:
        out["roofline"] = head["roofline"]
    if "fp64" in recs and head_name != "fp64":
        out["fp64"] = recs["fp64"]
        out["mixed_over_fp64"] = head["value"] / recs["fp64"]["value"]
    if not args.no_cpu_baseline:
        print("timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_side)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
