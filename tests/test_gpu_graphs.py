"""Captured DDM applications (HIP graphs) against eager launches.

With graphs on, a DDM application applied a second time with the same arrays
and column count is captured and replayed from then on.  Every replay must
equal the eager launches bit for bit: replays are interleaved with other
eager work of the library and synchronizations, and each is checked; the
results are also held to the oracle (FP64 DDM 1e-10, solves 1e-8)."""

import sys

import numpy as np
import pytest

import oracle as O
from paper_2003_02585_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_02585_amd import hdsw
    return hdsw


def _ctx(H, kap, h, P, W, **opt):
    ctx = H.hdsw_setup(kap, h, P, W, H.hdsw_default_options(**opt),
                       stream=torch.cuda.current_stream().cuda_stream)
    H.hdsw_factor(ctx)
    return ctx


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_replayed_applications_equal_eager(H, prec, dim):
    if dim == 2:
        N, W, P, pml = 48, 8, (3, 3), 1e-16
        h = 1.0 / N
        kap = wl.two_layer_kappa((N, N), h, 2 * np.pi / (10 * h), 3 * np.pi / (10 * h), 0.37)
        f = wl.sources((N, N), h, wl.random_positions(3, 2, 5, 4 * h, 1 - 4 * h), 2 * h)
        rounds = 2
    else:
        N, W, P, pml = 12, 3, (2, 2, 2), 1e-4
        h = 1.0 / N
        kap = wl.constant_kappa((N,) * 3, 2 * np.pi / (6 * h))
        f = wl.sources((N,) * 3, h, wl.random_positions(2, 3, 5, 0.2, 0.8), 2 * h)
        rounds = 1
    prob = O.Problem(kap, h, W, pml_R=pml)
    part = O.Partition(prob, P)
    b = np.stack([O.global_rhs(prob, fi) for fi in f])
    oref = [O.ddm_apply(prob, part, bi, rounds=rounds) for bi in b]
    _say(f"graph replay {dim}D {prec}")
    p = H.HDSW_FP64 if prec == "fp64" else H.HDSW_MIXED
    out = {}
    for graphs in (0, 1):
        ctx = _ctx(H, kap, h, P, W, precision=p, rounds=rounds, pml_R=pml, graphs=graphs)
        try:
            r = torch.from_numpy(b).cuda()
            z = torch.zeros_like(r)
            ft = torch.from_numpy(f).cuda()
            zs, xs = [], []
            for rep in range(4):
                z.fill_(7.0)
                H.hdsw_apply_precond(ctx, r, z, r.shape[0])      # eager, capture, replay, replay
                zs.append(z.cpu().numpy())
                # other eager work of the library between replays
                rr = torch.zeros_like(r)
                H.hdsw_residual(ctx, r, z, rr, r.shape[0])
                torch.cuda.synchronize()
            for rep in range(3):
                xt = torch.zeros_like(ft)
                H.hdsw_solve(ctx, ft, xt, ft.shape[0])             # refinement: replays inside
                xs.append(xt.cpu().numpy())
            out[graphs] = (zs, xs)
        finally:
            H.hdsw_destroy(ctx)
    ze, xe = out[0]
    zg, xg = out[1]
    for rep in range(4):
        assert np.array_equal(ze[rep], ze[0])
        assert np.array_equal(zg[rep], ze[0]), f"application {rep} differs from eager"
    for rep in range(3):
        assert np.array_equal(xg[rep], xe[0]), f"solve {rep} differs from eager"
    e = max(np.linalg.norm(z - o) / np.linalg.norm(o) for z, o in zip(ze[0], oref))
    _say(f"  rel diff vs oracle DDM {e:.3e}")
    assert e < (1e-10 if prec == "fp64" else 2e-4)


def test_replayed_gmres_equals_eager(H):
    N, W, P = 64, 16, (4, 4)
    h = 1.0 / N
    kap = wl.two_layer_kappa((N, N), h, 2 * np.pi / (10 * h), 3 * np.pi / (10 * h), 0.37)
    f = wl.sources((N, N), h, wl.random_positions(2, 2, 9, 4 * h, 1 - 4 * h), 2 * h)
    prob = O.Problem(kap, h, W)
    ug = O.solve_global(prob, np.stack([O.global_rhs(prob, fi) for fi in f]))
    sl = prob.interior_slice()
    _say("graph replay GMRES(20)")
    out = {}
    for graphs in (0, 1):
        ctx = _ctx(H, kap, h, P, W, precision=H.HDSW_MIXED, rounds=2, gmres_m=20,
                   tol=1e-11, max_iter=40, graphs=graphs)
        try:
            ft = torch.from_numpy(f).cuda()
            xs = []
            for rep in range(3):
                xt = torch.zeros_like(ft)
                H.hdsw_solve(ctx, ft, xt, 2)
                xs.append(xt.cpu().numpy())
            out[graphs] = xs
        finally:
            H.hdsw_destroy(ctx)
    for rep in range(3):
        assert np.array_equal(out[1][rep], out[0][0])
    e = max(np.linalg.norm(x - u[sl]) / np.linalg.norm(u[sl]) for x, u in zip(out[1][2], ug))
    _say(f"  rel err vs global solution {e:.3e}")
    assert e < 1e-8


def test_kernel_timing_runs_eager_with_graphs_on(H):
    # kernel-class timing needs per-launch events, which a graph's replay
    # cannot provide: with timing on the applications run eagerly, results
    # unchanged, and every launch is counted
    N, W, P = 48, 8, (3, 3)
    h = 1.0 / N
    kap = wl.constant_kappa((N, N), 2 * np.pi / (10 * h))
    f = wl.sources((N, N), h, wl.random_positions(2, 2, 5, 4 * h, 1 - 4 * h), 2 * h)
    prob = O.Problem(kap, h, W)
    b = np.stack([O.global_rhs(prob, fi) for fi in f])
    _say("timing with graphs on")
    ctx = _ctx(H, kap, h, P, W, precision=H.HDSW_MIXED, graphs=1)
    try:
        r = torch.from_numpy(b).cuda()
        z = torch.zeros_like(r)
        outs = []
        for rep in range(3):
            H.hdsw_apply_precond(ctx, r, z, 2)
            outs.append(z.cpu().numpy())
        H.hdsw_timing_enable(ctx, True)
        for rep in range(3):
            H.hdsw_apply_precond(ctx, r, z, 2)
            outs.append(z.cpu().numpy())
        ms, n, fl, by = H.hdsw_timing_get(ctx, H.KT_SOLVE)
        H.hdsw_timing_enable(ctx, False)
        H.hdsw_apply_precond(ctx, r, z, 2)
        outs.append(z.cpu().numpy())
    finally:
        H.hdsw_destroy(ctx)
    assert n == 6 and ms > 0
    for o in outs:
        assert np.array_equal(o, outs[0])


def test_recording_beside_a_factorizing_thread(H):
    # A worker thread sets up, factors and destroys contexts (allocations,
    # frees, blocking copies) while the main thread keeps recording and
    # replaying DDM applications of another context, each with new arrays
    # (a new graph per pair).  Neither side may fail, and every replay
    # equals the eager result of the same input bit for bit.
    import threading
    N, W, P = 64, 8, (4, 4)
    h = 1.0 / N
    kap = wl.constant_kappa((N, N), 2 * np.pi / (10 * h))
    f = wl.sources((N, N), h, wl.random_positions(2, 2, 9, 4 * h, 1 - 4 * h), 2 * h)
    prob = O.Problem(kap, h, W)
    b = torch.from_numpy(np.stack([O.global_rhs(prob, fi) for fi in f])).cuda()
    _say("graph recording beside a factorizing thread")
    ref_ctx = _ctx(H, kap, h, P, W, precision=H.HDSW_MIXED, graphs=0)
    ctx = _ctx(H, kap, h, P, W, precision=H.HDSW_MIXED, graphs=1)
    errors, done, factored = [], threading.Event(), [0]

    def worker():
        try:
            s = torch.cuda.Stream()
            k2 = wl.two_layer_kappa((N, N), h, 2 * np.pi / (10 * h), 3 * np.pi / (10 * h), 0.53)
            while not done.is_set():
                c = H.hdsw_setup(k2, h, P, W, H.hdsw_default_options(precision=H.HDSW_MIXED),
                                 stream=s.cuda_stream)
                try:
                    H.hdsw_factor(c)
                    H.hdsw_batch_reserve(c, 2)
                finally:
                    H.hdsw_destroy(c)
                factored[0] += 1
        except Exception as e:      # reported by the main thread
            errors.append(e)

    t = threading.Thread(target=worker)
    t.start()
    try:
        zref = torch.zeros_like(b)
        H.hdsw_apply_precond(ref_ctx, b, zref, 2)
        it = 0
        while (it < 12 or factored[0] < 3) and it < 400 and not errors:
            it += 1
            r = b.clone()
            z = torch.zeros_like(b)
            for _ in range(3):               # eager, recorded, replayed
                H.hdsw_apply_precond(ctx, r, z, 2)
                torch.cuda.synchronize()
                assert torch.equal(z, zref), it
    finally:
        done.set()
        t.join()
        H.hdsw_destroy(ctx)
        H.hdsw_destroy(ref_ctx)
    _say(f"  {it} recorded applications beside {factored[0]} factorizations")
    assert not errors, errors
    assert factored[0] >= 3
