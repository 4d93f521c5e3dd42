"""Benchmark: unknowns/s to factor and solve to relative residual 1e-10, the
mixed-precision form against the float64 form, on one MI355X.

Workload (default, --workload batch): 256 independent 2D upwind
convection-diffusion systems (sides uniform in [64, 512], Peclet uniform in
[1, 100], random direction; 26.6 M unknowns in total), leaves of 64, eps 1e-3,
one right-hand side each, right-preconditioned GMRES(30) to 1e-10 per system.
Systems are factored together with hs_factor_batch in groups whose measured
device footprint fits the memory budget; one step = every group's
hs_factor_batch + hs_gmres + hs_free, with the CSR matrices and right-hand
sides already resident in HBM.  value = unknowns * steps / seconds of the
mixed form (float32 blocks and records on the fine levels, Schur products on
the bfloat16 units, float64 coarse levels and Krylov vectors); the float64
form is timed the same way (min(steps, 3) steps) and reported beside it.

Also reported:
  * roofline: the pivot-block kernel on the float32 levels (k_pivot<true,
    float>, the kernel with the most GPU time in the mixed step), its
    algorithmic flops per launch over its average launch time (HIP events
    recorded on the library's stream around its launches inside the timed
    steps) against the FP64 peak (its arithmetic runs in float64);
  * cpu_baseline: the CPU oracle (plain numpy, FP64) on the 40 smallest of the
    same 256 systems, factor + GMRES(30) to 1e-10 each.

Other workloads: --workload poisson64 (3D Poisson 64^3, eps 1e-4, PCG for 8
RHS), --workload vcd128 (3D lognormal diffusion 128^3, eps 1e-3, PCG),
--workload serve (a Poisson stream of solve requests through the library's
request loop, p50 / p99 latency), --workload paper (the paper's Sec. 5.1
experiment: Poisson and quantized high-contrast variable-coefficient Poisson,
rank by an eps sweep or fixed K = 8 / 16, CG to 1e-12).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms both|mixed|fp64]
                       [--workload batch|poisson64|vcd128|serve] [--batch-count 256] [--budget-gb 200]
                       [--fp64-steps S] [--profile] [--no-cpu-baseline]
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

METRIC = "unknowns/s factor+solve to 1e-10 residual, mixed vs FP64; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # 256 CUs x 4 SIMDs x 16 lanes x 2 (fma) x 2.4 GHz; FP64 matrix cores: the same
PROFILES = os.path.join(ROOT, "profiles")
FAMILIES = ["gram", "pivot", "pivot_f32", "fill", "nbr", "schur", "schur_f32", "merge", "apply", "spmv", "dense",
            "host_symbolic", "host_plan", "host_upload", "host_alloc", "host_sync", "host_solve_plan"]


def _section(name, a, b):
    with open(os.path.join(ROOT, "paper_1712_07297_amd", "csrc", name)) as fh:
        text = fh.read()
    i = text.index(a)
    return text[i : text.index(b, i)]


def kernel_source_digest(kernel: str) -> str:
    """Digest of a kernel's source: its section of k_factor.hip and the
    device_common.h routines it is built on."""
    h = hashlib.sha256()
    if kernel == "schur":
        h.update(_section("k_factor.hip", "// " + "=" * 60 + " Schur update", "// " + "=" * 64 + " assembly").encode())
        h.update(_section("device_common.h", "// " + "-" * 60 + " MFMA tile core",
                          "// " + "-" * 60 + " cooperative GEMM").encode())
    else:  # pivot: the kernel and every routine of the header but the BF16 tile (not used by it)
        h.update(_section("k_factor.hip", "// " + "=" * 62 + " pivot kernel",
                          "// " + "=" * 50 + " pivoted Householder QR").encode())
        with open(os.path.join(ROOT, "paper_1712_07297_amd", "csrc", "device_common.h")) as fh:
            text = fh.read()
        bf16 = _section("device_common.h", "// " + "-" * 49 + " BF16 tile core", "// " + "-" * 60 + " cooperative GEMM")
        h.update(text.replace(bf16, "").encode())
    return h.hexdigest()[:16]


def measured_traffic(profile: str, kernel: str, key: str):
    """HBM bytes per launch from a committed FETCH_SIZE / WRITE_SIZE summary
    (profiles/<profile>), or None when the kernel's source changed since."""
    try:
        with open(os.path.join(PROFILES, profile)) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = dict(line.split(":", 1) for line in text.splitlines() if ":" in line and not line.startswith(("#", "|", " ")))
    if vals.get("kernel_source_digest", "").strip() != kernel_source_digest(kernel):
        return None
    v = vals.get(key)
    return float(v) if v is not None else None


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info

        return max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline_batch(probs, count: int = 40):
    """The oracle (plain numpy FP64) on the `count` smallest systems of the
    benchmarked batch: factor + GMRES(30) to 1e-10 each."""
    import oracle as O

    idx = sorted(range(len(probs)), key=lambda i: (probs[i].A.n, i))[:count]
    t0 = time.perf_counter()
    nsum = 0
    for i in idx:
        p = probs[i]
        fo = O.factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.leaf, p.eps, False)
        _, it, rel = O.gmres(p.A.row_ptr, p.A.col_idx, p.A.val, p.B[:, 0], lambda R: O.solve(fo, R), p.tol, 300, 30)
        assert rel <= p.tol
        nsum += p.A.n
    dt = time.perf_counter() - t0
    sides = sorted(probs[i].dims[0] for i in idx)
    return {
        "value": nsum / dt,
        "unit": "unknowns/s",
        "cores": int(_blas_threads()),
        "kind": "oracle",
        "sample": f"the {count} smallest of the same {len(probs)} systems (sides {sides[0]}..{sides[-1]}, {nsum} "
                  f"unknowns), leaf 64, eps 1e-3, factor + GMRES(30) to 1e-10 each: {dt:.1f} s",
    }


def cpu_baseline_poisson(side: int = 24):
    """The oracle on a side^3 Poisson sample of the 64^3 workload family:
    factor + PCG for 8 RHS to 1e-10."""
    import oracle as O
    from workloads import config2

    p = config2(side=side, nrhs=8)
    t0 = time.perf_counter()
    fo = O.factor(p.A.row_ptr, p.A.col_idx, p.A.val, p.dims, p.leaf, p.eps, True)
    X, it, rel = O.pcg(p.A.row_ptr, p.A.col_idx, p.A.val, p.B, lambda R: O.solve(fo, R), p.tol, 200)
    dt = time.perf_counter() - t0
    assert rel.max() <= p.tol
    return {
        "value": p.A.n / dt,
        "unit": "unknowns/s",
        "cores": int(_blas_threads()),
        "kind": "oracle",
        "sample": f"3D Poisson {side}^3 (N={p.A.n}), leaf 64, eps 1e-4, 8 RHS, PCG to 1e-10: one factor+solve "
                  f"in {dt:.1f} s (a smaller input of the same family)",
    }


def roofline_from(P, family, kernel_label, bound, traffic=None):
    """Roofline record of one kernel family timed by the library's events."""
    r = P.profile_read(family)
    if r["launches"] == 0 or r["seconds"] <= 0:
        return None
    out = {"kernel": kernel_label, "bound": bound}
    if bound == "hbm":
        achieved = r["bytes"] / r["seconds"] / 1e9
        out.update({"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS})
    else:
        achieved = r["flops"] / r["seconds"] / 1e12
        out.update({"achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP64_PEAK_TFLOPS})
    out.update({
        "traffic": traffic,
        "launches": r["launches"],
        "avg_launch_ms": r["seconds"] / r["launches"] * 1e3,
        "algorithmic_flops_per_launch": r["flops"] / r["launches"],
        "algorithmic_bytes_per_launch": r["bytes"] / r["launches"],
        "achieved_tflops": r["flops"] / r["seconds"] / 1e12,
        "achieved_gbs": r["bytes"] / r["seconds"] / 1e9,
    })
    return out


def measure_apply(P, torch, idx, sys_dev, rhs, precision, reps=5):
    """One application of the factor (hs_solve, one right-hand side per
    system: the forward and backward sweeps of Alg. 2) on the first group,
    outside the timed steps: the records' algorithmic bytes (every stored
    T_L', T_R', E_L, E_R element read once) over the time per solve."""
    F = P.Factor.batch([sys_dev[i] for i in idx], 1e-3, 64, symmetric=0, precision=precision)
    B = torch.cat([rhs[i] for i in idx]).reshape(1, -1)
    X = torch.empty_like(B)
    F.solve(B, X)  # captures the sweeps
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        F.solve(B, X)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    nbytes = F.info().factor_bytes
    F.free()
    return {"bytes_per_solve": nbytes, "ms_per_solve": ms, "achieved_GBps": nbytes / ms / 1e6,
            "frac_of_hbm": nbytes / ms / 1e6 / 8000.0, "systems": len(idx)}


def run_batch(args):
    """The batched convection-diffusion workload, mixed and float64 forms."""
    import torch

    import paper_1712_07297_amd as P
    from workloads import config4_batch

    dev = torch.device("cuda:0")
    P.lib()
    P.use_torch_allocator(args.allocator == "torch")
    t0 = time.perf_counter()
    probs = config4_batch(count=args.batch_count)
    ns = [p.A.n for p in probs]
    ntot = int(sum(ns))
    sys_dev = [(torch.tensor(p.A.row_ptr, device=dev), torch.tensor(p.A.col_idx, device=dev),
                torch.tensor(p.A.val, device=dev), p.dims) for p in probs]
    rhs = [torch.tensor(np.ascontiguousarray(p.B[:, 0]), device=dev) for p in probs]
    torch.cuda.synchronize()
    print(f"batch: {len(probs)} systems, {ntot} unknowns generated and uploaded in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    budget = args.budget_gb * 1e9
    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024 // 8, dtype=torch.float64, device=dev)  # 64 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    def run_group(idx, precision):
        F = P.Factor.batch([sys_dev[i] for i in idx], 1e-3, 64, symmetric=0, precision=precision)
        B = torch.cat([rhs[i] for i in idx]).reshape(1, -1)
        X, it, rel, ok = F.gmres(B, 1e-10, 300, 30)
        info = F.info()
        F.free()
        return X, it, float(np.max(rel)), ok, info

    out_forms = {}
    forms = {"both": [P.HS_MIXED, P.HS_FP64], "mixed": [P.HS_MIXED], "fp64": [P.HS_FP64]}[args.forms]
    for prec in forms:
        name = "mixed" if prec == P.HS_MIXED else "fp64"
        head = prec == forms[0]
        steps = args.steps if head else max(1, min(args.steps, args.fp64_steps))
        warmup = args.warmup if head else min(args.warmup, 1)
        # footprint per unknown from a calibration group of the first systems
        cal = list(range(min(8, len(probs))))
        info = run_group(cal, prec)[4]
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

        def step(record):
            results = [run_group(g, prec) for g in groups]
            for g, (X, it, rel, ok, info) in zip(groups, results):
                if record is not None:
                    record["its"].append(it)
                    record["rels"].append(rel)
                    record["oks"].append(ok)
                    record["peaks"].append(info.peak_device_bytes)
                    record["flops"] += info.factor_flops
                    record["X"].append((g, X))

        for w in range(warmup):
            step(None)
            print(f"batch {name}: warmup step {w + 1}/{warmup} done", file=sys.stderr, flush=True)
        pivot_family = "pivot_f32" if prec == P.HS_MIXED else "pivot"
        P.profile_reset()
        P.profile_select("" if args.profile else pivot_family)
        P.profile_enable(True)
        rec = {"its": [], "rels": [], "oks": [], "peaks": [], "flops": 0.0, "X": []}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for st in range(steps):
            rec["X"] = []
            step(rec)
            print(f"batch {name}: timed step {st + 1}/{steps} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        P.profile_enable(False)
        if args.profile:
            prof = {f: round(P.profile_read(f)["seconds"] / steps, 4) for f in FAMILIES}
            print(f"batch {name}: seconds per step by family {json.dumps(prof)}", file=sys.stderr, flush=True)
        label = ("k_pivot<true, float>" if prec == P.HS_MIXED else "k_pivot<true, double>") + \
            " (pivot-block LU, rank, complement, F_ff; Eqs. lra, scaling, elim)"
        traffic = measured_traffic("k_pivot_hbm_traffic_batch_convdiff256.md", "pivot",
                                   f"traffic_bytes_per_launch_{'float' if prec == P.HS_MIXED else 'double'}")
        roof = roofline_from(P, pivot_family, label, "alu", traffic)
        P.profile_select("")
        P.profile_reset()
        torch.cuda.empty_cache()  # hand cached blocks back before the next allocations
        apply = measure_apply(P, torch, groups[0], sys_dev, rhs, prec)
        print(f"batch {name}: apply {json.dumps(apply)}", file=sys.stderr, flush=True)
        # independent check of every system's final residual (device SpMV by torch, FP64)
        relcheck = 0.0
        for g, X in rec["X"]:
            x = X.reshape(-1)
            off = 0
            for i in g:
                rp, ci, va, _ = sys_dev[i]
                A_t = torch.sparse_csr_tensor(rp, ci.to(torch.int64), va, size=(ns[i], ns[i]))
                xi = x[off : off + ns[i]]
                r = rhs[i] - A_t @ xi
                relcheck = max(relcheck, (torch.linalg.norm(r) / torch.linalg.norm(rhs[i])).item())
                off += ns[i]
        out_forms[name] = {
            "value": ntot / dt,
            "ms_per_step": dt * 1e3,
            "steps": steps,
            "groups": len(groups),
            "gmres_iterations_max": int(max(rec["its"])),
            "relres_max": float(max(rec["rels"])),
            "relres_check": relcheck,
            "converged": bool(all(rec["oks"])) and max(rec["rels"]) <= 1e-10 and relcheck <= 1.01e-10,
            "peak_device_gb": float(max(rec["peaks"])) / 1e9,
            "factor_gflop_per_step": rec["flops"] / steps / 1e9,
            "apply": apply,
            "roofline": roof,
        }
    head_name = "mixed" if "mixed" in out_forms else "fp64"
    head = out_forms[head_name]
    out = {
        "metric": METRIC,
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
            "workload": f"batch of {len(probs)} 2D upwind convection-diffusion systems (sides 64..512, Peclet 1..100, "
                        f"N total {ntot}), leaf 64, eps 1e-3, hs_factor_batch + GMRES(30) to 1e-10 per system, "
                        "1 RHS each",
            "form": head_name,
            "allocator": "torch caching allocator" if args.allocator == "torch" else "HIP stream-ordered pool",
            **{k: v for k, v in head.items() if k not in ("value", "ms_per_step", "roofline")},
        },
    }
    if head.get("roofline"):
        out["roofline"] = head["roofline"]
    if "fp64" in out_forms and head_name != "fp64":
        out["fp64"] = out_forms["fp64"]
        out["mixed_over_fp64"] = head["value"] / out_forms["fp64"]["value"]
    if not args.no_cpu_baseline:
        print("timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_batch(probs)
    print(json.dumps(out))


def run_single(args):
    """One large system: 3D Poisson 64^3 (poisson64, PCG for 8 RHS) or 3D
    lognormal diffusion 128^3 (vcd128, PCG for 1 RHS); mixed and float64."""
    import torch

    import paper_1712_07297_amd as P
    from workloads import config2, config3

    dev = torch.device("cuda:0")
    if args.workload == "poisson64":
        p = config2(side=args.side, nrhs=args.nrhs)
        label = (f"3D 7-point Poisson {args.side}^3 (N={p.A.n}), leaf 64, eps 1e-4, PCG preconditioner, "
                 f"{args.nrhs} RHS to relative residual 1e-10")
    else:
        p = config3(side=args.side if args.side != 64 else 128)
        label = (f"3D finite-volume diffusion {p.dims[0]}^3 (N={p.A.n}), coefficients exp(g), g Gaussian, sigma 2, "
                 "correlation 8 cells, leaf 64, eps 1e-3, PCG preconditioner, 1 RHS to relative residual 1e-10")
    n = p.A.n
    rp = torch.tensor(p.A.row_ptr, device=dev)
    ci = torch.tensor(p.A.col_idx, device=dev)
    va = torch.tensor(p.A.val, device=dev)
    B = torch.tensor(np.ascontiguousarray(p.B.T), device=dev)  # (nrhs, n) = column-major n x nrhs
    X = torch.empty_like(B)
    if args.copy_probe:  # three plain copies of 64 MiB: the counter calibration
        src = torch.ones(64 * 1024 * 1024 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        del src, dst
    torch.cuda.synchronize()
    forms = {"both": [P.HS_MIXED, P.HS_FP64], "mixed": [P.HS_MIXED], "fp64": [P.HS_FP64]}[args.forms]
    recs = {}
    for prec in forms:
        name = "mixed" if prec == P.HS_MIXED else "fp64"
        split = {"factor": 0.0, "solve": 0.0}
        torch.cuda.empty_cache()  # the previous form's cached blocks back to the device

        def step():
            t0 = time.perf_counter()
            F = P.Factor(rp, ci, va, p.dims, p.eps, p.leaf, symmetric=1, precision=prec)
            t1 = time.perf_counter()
            _, it, rel, ok = F.pcg(B, p.tol, 300, X=X)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            split["factor"] += t1 - t0
            split["solve"] += t2 - t1
            info = F.info()
            F.free()
            return it, rel, ok, info

        try:
            for w in range(args.warmup):
                step()
                print(f"{name}: warmup step {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
        except P.HsError as e:  # a form that does not fit is reported, not timed
            print(f"{name}: {e}", file=sys.stderr, flush=True)
            recs[name] = {"error": str(e)}
            continue
        fam = "schur_f32" if prec == P.HS_MIXED else "schur"
        P.profile_reset()
        P.profile_select("" if args.profile else fam)
        P.profile_enable(True)
        torch.cuda.synchronize()
        split["factor"] = split["solve"] = 0.0
        t0 = time.perf_counter()
        its, rels, oks, info = [], [], [], None
        for k in range(args.steps):
            it, rel, ok, info = step()
            print(f"{name}: timed step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
            its.append(it)
            rels.append(float(rel.max()))
            oks.append(ok)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        P.profile_enable(False)
        if args.profile:
            prof = {f: round(P.profile_read(f)["seconds"] / args.steps, 4) for f in FAMILIES}
            print(f"{name}: seconds per step by family {json.dumps(prof)}", file=sys.stderr, flush=True)
        traffic = None
        if args.workload == "poisson64" and args.side == 64 and args.nrhs == 8:
            traffic = measured_traffic("k_schur_hbm_traffic_poisson64.md", "schur",
                                       f"traffic_bytes_per_launch_{'float' if prec == P.HS_MIXED else 'double'}")
        roof = roofline_from(P, fam, f"k_schur<{'float' if prec == P.HS_MIXED else 'double'}> "
                                     "(Schur-complement update, Eq. elim)", "hbm", traffic)
        P.profile_select("")
        P.profile_reset()
        A_t = torch.sparse_csr_tensor(rp, ci.to(torch.int64), va, size=(n, n))
        R = B.T - (A_t @ X.T)
        relres = (torch.linalg.norm(R, dim=0) / torch.linalg.norm(B.T, dim=0)).max().item()
        recs[name] = {
            "value": n * args.steps / dt,
            "ms_per_step": dt / args.steps * 1e3,
            "factor_ms": split["factor"] / args.steps * 1e3,
            "solve_ms": split["solve"] / args.steps * 1e3,
            "pcg_iterations": its,
            "relres_max": max(rels),
            "relres_check": relres,
            "converged": all(oks) and relres <= p.tol * 1.01,
            "levels": info.nlevels,
            "colour_batches": info.ncolors_total,
            "factor_gflop": info.factor_flops / 1e9,
            "factor_bytes_records": info.factor_bytes,
            "peak_device_gb": info.peak_device_bytes / 1e9,
            "roofline": roof,
        }
    ok_forms = [k for k in ("mixed", "fp64") if k in recs and "error" not in recs[k]]
    if not ok_forms:
        raise SystemExit("no form of the workload fits: " + json.dumps(recs))
    head_name = ok_forms[0]
    head = recs[head_name]
    out = {
        "metric": METRIC,
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
        "config": {"workload": label, "form": head_name,
                   **{k: v for k, v in head.items() if k not in ("value", "ms_per_step", "roofline")}},
    }
    if head.get("roofline"):
        out["roofline"] = head["roofline"]
    if "fp64" in recs and head_name != "fp64":
        out["fp64"] = recs["fp64"]
        if "error" not in recs["fp64"]:
            out["mixed_over_fp64"] = head["value"] / recs["fp64"]["value"]
    if not args.no_cpu_baseline and args.workload == "poisson64":
        print("timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_poisson(args.cpu_side)
    print(json.dumps(out))


def run_paper(args):
    """The paper's Sec. 5.1 experiment at one grid size: 3D Poisson and
    variable-coefficient Poisson (quantized high-contrast field, 1e2 / 1e-2)
    with the rank chosen by eps (a sweep) or fixed (K = 8 and K = 16), each
    factorization used as the CG preconditioner to 1e-12; and the Helmholtz
    equation at 32 points per wavelength (side / 32 Hz) with the eps sweep
    and K = 32, as the preconditioner of GMRES(30) to 1e-3.  One right-hand
    side uniform on [-1, 1).  Reports iterations, factor and solve times and
    the coarse sizes for every setting."""
    import torch

    import paper_1712_07297_amd as P
    from workloads import helmholtz3d, poisson3d, rhs_uniform, vc_poisson3d

    dev = torch.device("cuda:0")
    side = args.side
    eps_sweep = [(e, 0) for e in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5)]
    problems = [
        ("poisson", poisson3d(side, side, side), "cg", 1e-12, eps_sweep + [(1e-12, 8), (1e-12, 16)]),
        ("vcpoisson", vc_poisson3d(np.random.default_rng(3), side), "cg", 1e-12,
         eps_sweep + [(1e-12, 8), (1e-12, 16)]),
        ("helmholtz", helmholtz3d(side), "gmres", 1e-3, eps_sweep + [(1e-12, 32)]),
    ]
    prec = P.HS_MIXED if args.forms == "mixed" else P.HS_FP64
    rows = []
    for name, A, solver, tol, settings in problems:
        rp = torch.tensor(A.row_ptr, device=dev)
        ci = torch.tensor(A.col_idx, device=dev)
        va = torch.tensor(A.val, device=dev)
        B = torch.tensor(rhs_uniform(np.random.default_rng(8), A.n, 1).T.copy(), device=dev)
        for eps, K in settings:
            best = None
            for rep in range(1 + max(0, args.warmup)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F = P.Factor(rp, ci, va, (side,) * 3, eps, 64, symmetric=1, fixed_rank=K, precision=prec)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                if solver == "cg":
                    X, it, rel, ok = F.pcg(B, tol, 1000)
                else:
                    X, it, rel, ok = F.gmres(B, tol, 1000, 30)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                info = F.info()
                F.free()
                if rep >= min(1, args.warmup):
                    best = (t1 - t0, t2 - t1, it, float(np.max(rel)), ok, info)
            tf, ts, it, rel, ok, info = best
            row = {"problem": name, "solver": solver, "tol": tol, "eps": eps, "fixed_rank": K,
                   "iterations": int(it), "relres": rel, "converged": bool(ok), "factor_ms": tf * 1e3,
                   "solve_ms": ts * 1e3, "unknowns_per_s": A.n / (tf + ts), "levels": info.nlevels,
                   "coarse_dofs_level1": int(info.coarse_dofs[0]), "factor_gflop": info.factor_flops / 1e9,
                   "record_gb": info.factor_bytes / 1e9, "peak_device_gb": info.peak_device_bytes / 1e9}
            rows.append(row)
            print(f"paper: {name} eps={eps:g} K={K}: {it} iterations, factor {tf * 1e3:.0f} ms, "
                  f"solve {ts * 1e3:.0f} ms, relres {rel:.1e}", file=sys.stderr, flush=True)
    head = rows[0]
    out = {
        "metric": METRIC,
        "value": head["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": args.warmup,
        "ms_per_step": head["factor_ms"] + head["solve_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == P.HS_FP64 else "f32 storage + bf16x3 MFMA Schur, f64 Krylov",
        "data": "synthetic",
        "config": {"workload": f"paper Sec. 5.1 sweep at {side}^3 (N={side ** 3}): 3D Poisson and quantized "
                               "high-contrast variable-coefficient Poisson (eps 1e-1..1e-5, fixed rank 8 / 16, CG "
                               "to 1e-12), Helmholtz at 32 points per wavelength (eps 1e-1..1e-5, fixed rank 32, "
                               "GMRES(30) to 1e-3), 1 RHS; value = the first row",
                   "sweep": rows},
    }
    print(json.dumps(out))


def run_serve(args):
    """The serving stream: Poisson arrivals of solve requests (60 % 3D
    lognormal diffusion, CG; 40 % 2D convection-diffusion, GMRES(30); 1-16
    right-hand sides; 30 % reuse an earlier operator), mixed form, served by
    the library's request loop.  The sustained capacity mu is the completion
    rate of a closed loop that keeps one request per worker in flight; the
    stream is then replayed at each load rho (arrival rate rho mu), each on a
    fresh server."""
    import torch

    import paper_1712_07297_amd as P
    from workloads import build_request_operator, serving_stream

    dev = torch.device("cuda:0")
    # the server admits work by the bytes its factorizations hold; blocks that a
    # caching allocator keeps after an eviction are invisible to that cap (and
    # cached per worker stream), so the serving runs take HIP's pool
    P.lib()
    P.use_torch_allocator(False)
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

    # warm-up: a few requests on a server of their own
    srv = make_server()
    for t in [submit(srv, i) for i in range(min(4, len(reqs)))]:
        srv.wait(t)
    srv.close()
    # sustained capacity: closed loop, one request per worker in flight
    cal = len(reqs) if args.calibrate <= 0 else min(args.calibrate, len(reqs))
    srv = make_server()
    inflight = []
    tc = time.perf_counter()
    for i in range(cal):
        if len(inflight) >= args.workers:
            srv.wait(inflight.pop(0))
        inflight.append(submit(srv, i))
    for t in inflight:
        srv.wait(t)
    mu = cal / (time.perf_counter() - tc)
    srv.close()
    print(f"serve: sustained capacity {mu:.2f} requests/s (closed loop over {cal} requests, {args.workers} in flight)",
          file=sys.stderr, flush=True)

    runs = []
    for rho in [float(x) for x in str(args.rho).split(",")]:
        lam = rho * mu
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
            if (i + 1) % 50 == 0:
                print(f"serve: rho {rho}: {i + 1}/{len(reqs)} submitted", file=sys.stderr, flush=True)
        results = [srv.wait(t)[1] for t in tickets]
        wall = time.perf_counter() - start
        st = srv.stats()
        srv.close()
        # a request that did not succeed: what it was, how the server ran it,
        # and the same request factored and solved alone
        failed = []
        for i, res in enumerate(results):
            if res["status"] == 0:
                continue
            r = reqs[i]
            rp, ci, va, dims, sym, n = ops[r.op_key]
            rec = {"request": i, "kind": r.kind, "side": r.side, "nrhs": r.nrhs, "status": int(res["status"]),
                   "iterations": int(res["iterations"]), "relres": float(res["relres"]),
                   "reused": int(res["reused"]), "batch_size": int(res["batch_size"])}
            try:
                F = P.Factor(rp, ci, va, dims, 1e-3, 64, symmetric=sym, precision=P.HS_MIXED)
                Xa, it_a, rel_a, ok_a = (F.pcg if sym else (lambda B_, t_, m_: F.gmres(B_, t_, m_, 30)))(rhs[i], 1e-10, 300)
                F.free()
                rec["alone"] = {"iterations": int(it_a), "relres": float(np.max(rel_a)), "converged": bool(ok_a)}
            except P.HsError as e:
                rec["alone"] = {"error": str(e)}
            failed.append(rec)
            print(f"serve: rho {rho}: request {i} did not succeed: {json.dumps(rec)}", file=sys.stderr, flush=True)
        runs.append({
            "rho": rho,
            "arrival_rate_per_s": lam,
            "unknowns_per_s": st["unknowns_per_s"],
            "requests_per_s": st["requests_per_s"],
            "p50_latency_s": st["p50_latency_s"],
            "p99_latency_s": st["p99_latency_s"],
            "mean_queue_s": st["mean_queue_s"],
            "wall_s": wall,
            "completed": st["completed"],
            "reused": st["reused"],
            "batches": st["batches"],
            "factored_ops": st["factored_ops"],
            "evictions": st["evictions"],
            "peak_held_gb": st["peak_held_bytes"] / 1e9,
            "max_relres": max(r["relres"] for r in results if r["status"] == 0),
            "failed": sum(1 for r in results if r["status"] != 0),
            "failed_status": sorted({int(r["status"]) for r in results if r["status"] != 0}),
            "failed_requests": failed,
            "converged": all(r["status"] == 0 for r in results) and max(r["relres"] for r in results) <= 1e-10,
        })
        print(f"serve: rho {rho}: {json.dumps(runs[-1])}", file=sys.stderr, flush=True)
    head = min(runs, key=lambda r: abs(r["rho"] - 0.8))
    out = {
        "metric": METRIC,
        "value": head["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": len(runs),
        "warmup": 1,
        "ms_per_step": head["wall_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage + bf16x3 MFMA Schur, f64 Krylov",
        "data": "synthetic",
        "config": {
            "workload": f"serving stream of {len(reqs)} requests ({len(ops)} operators): 60% 3D lognormal diffusion "
                        "(sides 32..96, CG), 40% 2D convection-diffusion (sides 256..1024, GMRES(30)), 1-16 RHS, "
                        "30% operator reuse, Poisson arrivals, eps 1e-3, tol 1e-10",
            "capacity_per_s": mu,
            "capacity_method": f"closed loop over {cal} requests, {args.workers} in flight",
            "rho": head["rho"],
            "cap_gb": args.cap_gb,
            "workers": args.workers,
            "runs": runs,
        },
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=3, help="timed steps of the float64 form (at most --steps)")
    ap.add_argument("--side", type=int, default=64)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--forms", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=24)
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--workload", choices=["batch", "poisson64", "vcd128", "serve", "paper"], default="batch")
    ap.add_argument("--requests", type=int, default=100, help="serve workload: requests in the stream")
    ap.add_argument("--rho", type=str, default="0.5,0.8,0.95",
                    help="serve workload: loads over the sustained capacity (comma-separated)")
    ap.add_argument("--cap-gb", type=float, default=200.0, help="serve workload: device memory cap")
    ap.add_argument("--workers", type=int, default=2, help="serve workload: batches in flight")
    ap.add_argument("--calibrate", type=int, default=0,
                    help="serve workload: requests of the closed-loop capacity run (0: the whole stream)")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--budget-gb", type=float, default=200.0, help="device memory per batched group")
    ap.add_argument("--allocator", choices=["torch", "hip"], default="torch",
                    help="device memory of the library: PyTorch's caching allocator or HIP's pool")
    ap.add_argument("--profile", action="store_true", help="per-family times (HIP events, host wall) to stderr")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args)
    elif args.workload == "serve":
        run_serve(args)
    elif args.workload == "paper":
        run_paper(args)
    else:
        run_single(args)


if __name__ == "__main__":
    main()
