"""The serving loop on the GPU: a Poisson mix of requests of several grid
sizes, subdomain sizes and media, with columns joining and leaving context
slots as they converge, gives for every request the same result as the
request solved alone (bit for bit: a column's arithmetic does not depend on
its neighbours), and those results reach the global PML solution of the
FP64 oracle."""

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
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_02585_amd import hdsw, serve
    return hdsw, serve


def _mix():
    # 10 requests over 5 keys, arrivals at 400 requests/s so that they
    # overlap; R up to 5 against a capacity of 3 slots per context
    return wl.request_stream(10, 400.0, seed=wl.SEED_BASE + 5, sizes=(128, 256),
                             subdomains=(32, 64), ppws=(10,), heights=(0.37,), rmax=5)


def test_mix_equals_alone_and_oracle(env):
    H, serve = env
    reqs_in = _mix()
    _say(f"serving mix: {[(r['key'], len(r['positions'])) for r in reqs_in]}")
    ex = serve.HipExecutor(cap_max=3, tol=1e-10)
    srv = serve.Server(ex, budget_bytes=4e9, tol=1e-10, max_iter=30, keep_results=True)
    reqs = srv.run(reqs_in)
    torch.cuda.synchronize()
    m = serve.metrics(srv, reqs)
    srv.close()
    _say(f"  metrics {m}")
    assert m["failed"] == 0
    assert all(r.hit is not None for r in reqs)
    assert max(x for r in reqs for x in r.rel) <= 1e-10

    # each request alone, from the same input: a fresh context, hdsw_solve
    # one column at a time
    for r in reqs:
        kap, h, P, W, rounds = wl.serve_kappa(r.key)
        N = kap.shape[-1]
        f = ex.sources(N, h, r.positions)
        torch.cuda.synchronize()
        opt = H.hdsw_default_options(precision=H.HDSW_MIXED, rounds=rounds, tol=1e-10)
        ctx = H.hdsw_setup(kap, h, P, W, opt,
                           stream=torch.cuda.current_stream().cuda_stream)
        try:
            H.hdsw_factor(ctx)
            alone = []
            for j in range(r.R):
                fj = f[j:j + 1].contiguous()
                xj = torch.zeros_like(fj)
                info, _ = H.hdsw_solve(ctx, fj, xj, 1)
                assert info[0][0] == r.iters[j]
                alone.append(xj.cpu().numpy()[0])
        finally:
            H.hdsw_destroy(ctx)
        mix = r.result.cpu().numpy()
        same = all(np.array_equal(mix[j], alone[j]) for j in range(r.R))
        _say(f"  request {r.rid} key {r.key} R={r.R} iters {r.iters} alone==mix {same}")
        assert same

    # the two smallest requests against the oracle's global solution
    small = sorted(reqs, key=lambda r: (r.key[0], r.R))[:2]
    for r in small:
        kap, h, P, W, rounds = wl.serve_kappa(r.key)
        N = kap.shape[-1]
        prob = O.Problem(kap, h, W)
        f = wl.sources((N, N), h, r.positions, 2 * h)
        b = np.stack([O.global_rhs(prob, fj) for fj in f])
        ug = O.solve_global(prob, b)
        sl = prob.interior_slice()
        mix = r.result.cpu().numpy()
        e = max(np.linalg.norm(mix[j] - ug[j][sl]) / np.linalg.norm(ug[j][sl])
                for j in range(r.R))
        _say(f"  request {r.rid} vs oracle global solution: {e:.3e}")
        assert e < 1e-8
