"""Autotuner of the kernels' launch parameters (hdsw_tuning_set).

For a factored context it times one DDM application (the hot path: block
solves and sweep steps of every subdomain, all right-hand-side columns)
under every candidate of the search space with device events on the
context's stream, keeps the fastest, and caches the choice in a JSON file
keyed by the shape that decides the kernels' performance:

    d<dim> ne<extended subdomain nodes per axis> P<subdomains> ops<distinct
    operators> <c64|c128> r<rounds>

(the number of columns it was tuned at is stored with the entry).  Search
space: 2D complex64 block solve with 8 or 16 columns per workgroup; 2D
sweep step with 2 or 4 row tiles per workgroup and 6/8/10 (complex64) or
3/4/5/6 (complex128) slices per register batch; 3D products with at most 8
columns through the streaming or the tiled kernel.  The row-tile split and
the 3D kernel form fix the order of partial sums, so a context keeps one
choice for every call (never one per column count), and a column's result
stays independent of the other columns of its batch.

python -m paper_2003_02585_amd.autotune --config layer2d [--precision mixed]
    tunes that workload's shape and writes the entry to tuning.json.
"""

import argparse
import itertools
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")


def shape_key(kappa_shape, P, W, precision_mixed, rounds, nops):
    """Cache key of a context (axes in x, y[, z] order)."""
    ne = [n // p + 2 * W for n, p in zip(reversed(kappa_shape), P)]
    return (f"d{len(ne)} ne{'x'.join(map(str, ne))} P{'x'.join(map(str, P))} ops{nops} "
            f"{'c64' if precision_mixed else 'c128'} r{rounds}")


def candidates(dim, mixed):
    """Every candidate of the search space for a context (dicts of
    hdsw_tuning fields)."""
    if dim == 2:
        ngs = (1, 2) if mixed else (1,)
        kbs = (6, 8, 10) if mixed else (3, 4, 5, 6)
        # complex128 four-wave workgroups with four row tiles need more than
        # half the register file at depths 5 and 6 (one workgroup per CU):
        # left out
        return [dict(solve_ng=ng, sweep_rw=rw, sweep_kb=kb, gemm_skinny=0, sweep_nw=nw,
                     sweep_sched=0)
                for ng, rw, kb, nw in itertools.product(ngs, (2, 4), kbs, (8, 4))
                if mixed or not (nw == 4 and rw == 4 and kb >= 5)]
    return [dict(solve_ng=0, sweep_rw=0, sweep_kb=0, gemm_skinny=s, sweep_nw=0, sweep_sched=0)
            for s in (1, 2)]


def time_application(H, torch, ctx, r, z, reps):
    """Median milliseconds of one DDM application (device events on the
    current stream, which is the context's stream)."""
    n = r.shape[0]
    for _ in range(2):                       # eager, then captured
        H.hdsw_apply_precond(ctx, r, z, n)
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        H.hdsw_apply_precond(ctx, r, z, n)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms))


def search(H, torch, ctx, r, dim, mixed, reps=5, log=None):
    """Times the built-in rules and every candidate on the context's data;
    leaves the fastest set on the context and returns the record."""
    z = torch.zeros_like(r)
    H.hdsw_tuning_set(ctx)                   # built-in rules
    default_ms = time_application(H, torch, ctx, r, z, reps)
    rows = []
    for cand in candidates(dim, mixed):
        H.hdsw_tuning_set(ctx, **cand)
        ms = time_application(H, torch, ctx, r, z, reps)
        rows.append((cand, ms))
        if log:
            log(f"  {cand}: {ms:.3f} ms")
    best, best_ms = min(rows, key=lambda t: t[1])
    if best_ms >= default_ms:
        best, best_ms = dict(solve_ng=0, sweep_rw=0, sweep_kb=0, gemm_skinny=0,
                             sweep_nw=0, sweep_sched=0), default_ms
    H.hdsw_tuning_set(ctx, **best)
    return dict(params=best, ms=best_ms, default_ms=default_ms, columns=int(r.shape[0]),
                candidates=[[c, round(m, 4)] for c, m in rows])


def load(path=CACHE):
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh).get("entries", {})


def save(entries, path=CACHE):
    with open(path, "w") as fh:
        json.dump({"version": 1, "entries": entries}, fh, indent=1, sort_keys=True)
        fh.write("\n")


def apply_cached(H, ctx, key, path=CACHE):
    """Sets the cached choice for `key` on the context; returns the entry or
    None (built-in rules stay)."""
    e = load(path).get(key)
    if e is not None:
        H.hdsw_tuning_set(ctx, **e["params"])
    return e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="layer2d")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--cache", default=CACHE)
    a = ap.parse_args()
    import torch
    from . import hdsw as H
    from . import workloads as wl
    w = wl.make(a.config)
    mixed = a.precision == "mixed"
    opt = H.hdsw_default_options(precision=H.HDSW_MIXED if mixed else H.HDSW_FP64,
                                 rounds=w["rounds"])
    ctx = H.hdsw_setup(w["kappa"], w["h"], w["P"], w["W"], opt,
                       stream=torch.cuda.current_stream().cuda_stream)
    try:
        H.hdsw_factor(ctx)
        _, nops, _ = H.hdsw_query(ctx)
        key = shape_key(w["kappa"].shape, w["P"], w["W"], mixed, w["rounds"], nops)
        # a dense b-space input (every subdomain active, as in every
        # refinement iteration after the first)
        gshape = tuple(n + 2 * w["W"] for n in w["kappa"].shape)
        rng = np.random.default_rng(1)
        r = rng.standard_normal((len(w["f"]),) + gshape) + 1j * rng.standard_normal(
            (len(w["f"]),) + gshape)
        rt = torch.from_numpy(r).cuda()
        print(f"tuning {key} at {rt.shape[0]} columns", flush=True)
        rec = search(H, torch, ctx, rt, w["kappa"].ndim, mixed, reps=a.reps,
                     log=lambda s: print(s, flush=True))
    finally:
        H.hdsw_destroy(ctx)
    entries = load(a.cache)
    entries[key] = rec
    save(entries, a.cache)
    print(f"{key}: best {rec['params']} {rec['ms']:.3f} ms, built-in rules "
          f"{rec['default_ms']:.3f} ms -> {a.cache}", flush=True)


if __name__ == "__main__":
    main()
