"""Benchmark: RHS-solves/s at relative error 1e-8 for the trace-transfer
diagonal sweeping DDM (Algorithm 2.1) as preconditioner of an FP64
iteration, mixed precision (complex64 factors and sweeps) vs the plain FP64
path, with p50/p99 solve latency.

Workload (default): 2D, 1024^2 interior nodes, k = 2 pi / (10 h) (10 points
per wavelength), PML 16 nodes, 8 x 8 subdomains of 128^2, 16 Gaussian point
sources (sigma = 2h) at seeded uniform positions; one round of four sweeps
per DDM application; FP64 refinement to ||b - S x|| / ||b|| <= tol.

One step = one hdsw_solve of the whole batch (factors resident, sources
resident in HBM).  value = nrhs * steps / timed seconds.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and the derived vector-ALU peaks:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s for
# non-packed FP32 or FP64 FMA; dense MFMA FP32 157.3, FP64 78.6 TFLOP/s.
PEAK_HBM_GBS = 8000.0
PEAK = {("alu", "f32"): 78.6, ("alu", "f64"): 78.6,
        ("mfma", "f32"): 157.3, ("mfma", "f64"): 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2d")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rhs", type=int, default=4)
    ap.add_argument("--dedup", type=int, default=1,
                    help="share factors of identical subdomain operators (0: one per subdomain)")
    ap.add_argument("--gmres-m", type=int, default=0, help="GMRES(m) instead of refinement")
    ap.add_argument("--rounds", type=int, default=None, help="rounds of sweeps per DDM")
    ap.add_argument("--hbm-budget-gb", type=float, default=0.0)
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 comparison path (factors too large for both)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy 5 times (HBM counter scale)")
    return ap.parse_args()


def run_path(H, torch, w, precision, steps, warmup, tol, timing, a):
    stream = torch.cuda.current_stream().cuda_stream
    opt = H.hdsw_default_options(precision=precision, tol=tol, rounds=w["rounds"],
                                 max_iter=40, dedup=a.dedup, gmres_m=a.gmres_m,
                                 hbm_budget=int(a.hbm_budget_gb * (1 << 30)))
    ctx = H.hdsw_setup(w["kappa"], w["h"], w["P"], w["W"], opt, stream=stream)
    try:
        torch.cuda.synchronize()
        H.hdsw_timing_enable(ctx, True)
        t0 = time.perf_counter()
        H.hdsw_factor(ctx)
        torch.cuda.synchronize()
        t_factor = time.perf_counter() - t0
        kt_factor = H.hdsw_timing_get(ctx, 2)
        H.hdsw_timing_enable(ctx, False)
        f = torch.from_numpy(w["f"]).cuda()
        x = torch.zeros_like(f)
        nrhs = f.shape[0]
        info = None
        for _ in range(warmup):
            info, _ = H.hdsw_solve(ctx, f, x, nrhs)
        kt_all, t_all_solve, dom = None, None, None
        if timing:
            # one untimed solve with every kernel class timed: the kernel
            # table and the dominant class
            H.hdsw_timing_enable(ctx, True)
            for k in range(4):
                H.hdsw_timing_get(ctx, k)          # reset
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H.hdsw_solve(ctx, f, x, nrhs)
            torch.cuda.synchronize()
            t_all_solve = time.perf_counter() - t0
            kt_all = {k: H.hdsw_timing_get(ctx, k) for k in range(4)}
            dom = max((0, 1), key=lambda k: kt_all[k][0])
            # the timed steps carry events around the dominant class only
            H.hdsw_timing_enable(ctx, 1 << dom)
            for k in range(4):
                H.hdsw_timing_get(ctx, k)          # reset
        lat = []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            info, _ = H.hdsw_solve(ctx, f, x, nrhs)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
        total = time.perf_counter() - t_all
        kt = None
        if timing:
            kt = {k: H.hdsw_timing_get(ctx, k) for k in range(4)}
            H.hdsw_timing_enable(ctx, False)
        fb, nops, ws = H.hdsw_query(ctx)
        return dict(total=total, lat=lat, info=info, x=x.cpu().numpy(), t_factor=t_factor,
                    kt=kt, kt_all=kt_all, t_all_solve=t_all_solve, dom=dom,
                    factor_bytes=fb, nops=nops, ws=ws, nrhs=nrhs, kt_factor=kt_factor)
    finally:
        H.hdsw_destroy(ctx)


def cpu_baseline(w, iters, nsample):
    """The FP64 oracle as it stands, on a bounded sample: `nsample` RHS
    through one DDM application (Algorithm 2.1) plus the factorization, then
    scaled to RHS-solves/s with the iteration count the FP64 path needed."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    prob = O.Problem(w["kappa"], w["h"], w["W"])
    part = O.Partition(prob, w["P"])
    t0 = time.perf_counter()
    sol = O.SubdomainSolvers(part)
    t_fac = time.perf_counter() - t0
    b = O.global_rhs(prob, w["f"][0])
    S = O.global_operator(prob)
    t0 = time.perf_counter()
    for _ in range(nsample):
        O.ddm_apply(prob, part, b, rounds=w["rounds"], solvers=sol)
        S @ b.ravel()
    t_app = (time.perf_counter() - t0) / nsample
    per_rhs = t_app * max(iters, 1)
    return dict(value=1.0 / per_rhs, unit="RHS-solves/s", cores=int(cores), kind="oracle",
                sample=(f"{nsample} RHS x 1 DDM application (+ residual) of the same "
                        f"workload, {t_app:.2f} s each, scaled by the {iters} iterations "
                        f"the FP64 path needed; factorization {t_fac:.2f} s not counted"))


def factor_mfma(mixed, fp64):
    """Achieved rate of the factorization (8 n^3 flops per block and
    distinct operator) against the MFMA peak of its precision."""
    out = {}
    for name, r, peak in (("mixed", mixed, PEAK[("mfma", "f32")]),
                          ("fp64", fp64, PEAK[("mfma", "f64")])):
        if r is None:
            continue
        ms, n, fl, _ = r["kt_factor"]
        if n and ms > 0:
            ach = fl / (ms * 1e-3) / 1e12
            out[name] = {"ms": round(ms, 3), "achieved_TFLOPs": round(ach, 3),
                         "peak": peak, "frac": round(ach / peak, 4)}
    return out


def describe(a, w, nrhs):
    d = w["kappa"].ndim
    N = w["kappa"].shape[-1]
    P = "x".join(str(p) for p in w["P"])
    kmin, kmax = float(w["kappa"].min()), float(w["kappa"].max())
    ppw = 2 * np.pi / (kmin * w["h"])
    med = (f"constant k, {ppw:.0f} points per wavelength" if kmax == kmin else
           f"two-layer k, {ppw:.0f} points per wavelength below, k2/k1 = {kmax / kmin:.2f}")
    it = f"GMRES({a.gmres_m})" if a.gmres_m else "FP64 refinement"
    return (f"{a.config}: {d}D {N}^{d} interior, {P} subdomains, PML {w['W']}, {med}, "
            f"{nrhs} Gaussian sources, {w['rounds']} round(s) of sweeps per DDM, {it}")


def measured_traffic(a, dom):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary of this workload, when that summary was taken
    on the current kernel source (sha256 of mfma.hip); else None."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"pmc_{a.config}.md")
    src = os.path.join(ROOT, "paper_2003_02585_amd", "csrc", "mfma.hip")
    if not os.path.exists(path) or a.dedup != 1 or a.gmres_m or a.rounds is not None:
        return None
    txt = open(path).read()
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    m = re.search(r"source sha256: ([0-9a-f]{64})", txt)
    if not m or m.group(1) != h:
        return None
    key = "sweep_step" if dom == 1 else "block_solve"
    m = re.search(rf"traffic_bytes_per_launch\[{key}\]: ([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def copy_calibration(torch):
    """A plain device copy of known size, for scaling the HBM counters."""
    n = 512 << 20
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    x.fill_(1)
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "repeats": 5}))


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    if a.copy_calibration:
        copy_calibration(torch)
        return
    from paper_2003_02585_amd import hdsw as H
    from paper_2003_02585_amd import workloads as wl

    w = wl.make(a.config)
    if a.rounds is not None:
        w["rounds"] = a.rounds
    mixed = run_path(H, torch, w, H.HDSW_MIXED, a.steps, a.warmup, a.tol, True, a)
    fsteps = a.fp64_steps if a.fp64_steps is not None else max(1, a.steps // 2)
    fp64 = None if a.no_fp64 else run_path(H, torch, w, H.HDSW_FP64, fsteps, 1, a.tol, False, a)
    nrhs = mixed["nrhs"]
    value = nrhs * a.steps / mixed["total"]
    v64 = nrhs * fsteps / fp64["total"] if fp64 else None
    lat = np.array(mixed["lat"]) * 1e3
    # accuracy: mixed vs FP64 results (both iterated to the same tolerance)
    rel_mf = None
    if fp64:
        x1, x2 = mixed["x"], fp64["x"]
        rel_mf = max(np.linalg.norm(p - q) / np.linalg.norm(q) for p, q in zip(x1, x2))
    # kernel table from the solve with every class timed; roofline of the
    # dominant class from the HIP events of the timed steps
    kt_all, kt = mixed["kt_all"], mixed["kt"]
    if w["kappa"].ndim == 3:
        names = {0: "k_plane_rhs+k_cgemm (plane-block solve of every subdomain)",
                 1: "k_sweep_step (fused sweep step)"}
    else:
        names = {0: "k_solve_fwd+k_solve_bwd (batched block solve)",
                 1: "k_sweep_step (fused sweep step)"}
    peak = PEAK[("mfma", "f32")]
    def entry(t, total_s):
        ms, n, fl, by = t
        avg_ms = ms / max(n, 1)
        ach = (fl / max(n, 1)) / (avg_ms * 1e-3) / 1e12 if n else 0.0
        return {"share_of_step": round(ms / (1e3 * total_s), 4),
                "avg_launch_ms": round(avg_ms, 5), "launches": n,
                "achieved_TFLOPs": round(ach, 3),
                "algorithmic_flops_per_launch": fl / max(n, 1),
                "algorithmic_bytes_per_launch": by / max(n, 1)}
    kernels = {names[k]: entry(kt_all[k], mixed["t_all_solve"]) for k in (0, 1)}
    dom = mixed["dom"]
    d = entry(kt[dom], mixed["total"])
    kernels[names[dom]]["timed_steps"] = {k: d[k] for k in ("avg_launch_ms", "launches",
                                                             "achieved_TFLOPs")}
    roof = {"bound": "mfma", "achieved": d["achieved_TFLOPs"], "peak": peak, "unit": "TFLOP/s",
            "frac": round(d["achieved_TFLOPs"] / peak, 4),
            "traffic": measured_traffic(a, dom),
            "kernel": names[dom], "avg_launch_ms": d["avg_launch_ms"],
            "launches": d["launches"]}
    iters64 = max(i for i, _ in fp64["info"]) if fp64 else max(i for i, _ in mixed["info"])
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(w, iters64, a.cpu_sample_rhs)
    out = {
        "metric": "RHS-solves/s at rel err 1e-8, mixed vs FP64 sweep; p50/p99 solve latency",
        "value": round(value, 3), "unit": "RHS-solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(float(lat.mean()), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": describe(a, w, nrhs), "nrhs": nrhs, "tol": a.tol,
                   "rounds": w["rounds"], "dedup": a.dedup, "gmres_m": a.gmres_m,
                   "distinct_operators": mixed["nops"]},
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "fp64_value": round(v64, 3) if v64 else None,
        "speedup_mixed_vs_fp64": round(value / v64, 3) if v64 else None,
        "iters_mixed": [i for i, _ in mixed["info"]],
        "iters_fp64": [i for i, _ in fp64["info"]] if fp64 else None,
        "rel_residual_max": max(r for _, r in mixed["info"]),
        "rel_diff_mixed_vs_fp64": rel_mf,
        "factor_s": {"mixed": round(mixed["t_factor"], 3),
                     "fp64": round(fp64["t_factor"], 3) if fp64 else None},
        "roofline": roof, "kernels": kernels, "factor_mfma": factor_mfma(mixed, fp64),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
