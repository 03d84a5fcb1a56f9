"""GPU checks of the kernels' launch parameters (the autotuner's search
space): every candidate keeps the result within the method's parity bars
against the oracle, parameters that only regroup independent columns or
change batch depths leave results bit for bit unchanged, invalid values are
refused, and the search leaves its fastest candidate set."""

import sys

import numpy as np
import pytest

import oracle as O
from paper_2003_02585_amd import autotune as A
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


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_every_candidate_matches_the_oracle(H, prec):
    N, W, P = 64, 8, (4, 4)
    h = 1.0 / N
    kap = wl.two_layer_kappa((N, N), h, 2 * np.pi / (10 * h), 3 * np.pi / (10 * h), 0.37)
    f = wl.sources((N, N), h, wl.random_positions(20, 2, 3, 4 * h, 1 - 4 * h), 2 * h)
    prob = O.Problem(kap, h, W)
    part = O.Partition(prob, P)
    b = np.stack([O.global_rhs(prob, fi) for fi in f])
    sol = O.SubdomainSolvers(part)
    pick = [0, 9, 19]
    oref = [O.ddm_apply(prob, part, b[i], rounds=2, solvers=sol) for i in pick]
    mixed = prec == "mixed"
    _say(f"tuning candidates {prec}")
    ctx = H.hdsw_setup(kap, h, P, W, H.hdsw_default_options(
        precision=H.HDSW_MIXED if mixed else H.HDSW_FP64, rounds=2),
        stream=torch.cuda.current_stream().cuda_stream)
    try:
        H.hdsw_factor(ctx)
        r = torch.from_numpy(b).cuda()
        z = torch.zeros_like(r)
        for bad in (dict(solve_ng=3), dict(sweep_rw=3), dict(sweep_kb=7 if mixed else 8),
                    dict(gemm_skinny=5), dict(sweep_nw=2)):
            with pytest.raises(H.HdswError) as ei:
                H.hdsw_tuning_set(ctx, **bad)
            assert ei.value.status == H.HDSW_EINVAL
        by_rw = {}
        for cand in A.candidates(2, mixed):
            H.hdsw_tuning_set(ctx, **cand)
            assert H.hdsw_tuning_get(ctx) == cand
            H.hdsw_apply_precond(ctx, r, z, 20)
            got = z.cpu().numpy()
            e = max(np.linalg.norm(got[i] - o) / np.linalg.norm(o) for i, o in zip(pick, oref))
            assert e < (2e-4 if mixed else 1e-10), (cand, e)
            # columns per workgroup and batch depth never change a result
            split = (cand["sweep_rw"], cand["sweep_nw"])
            if split in by_rw:
                assert np.array_equal(got, by_rw[split]), cand
            else:
                by_rw[split] = got
    finally:
        H.hdsw_destroy(ctx)


def test_search_sets_its_fastest_candidate(H):
    w = wl.make("c2d", N=256, P=4, nrhs=4)
    _say("autotune search at 256^2, 4x4, 4 columns")
    ctx = H.hdsw_setup(w["kappa"], w["h"], w["P"], w["W"], H.hdsw_default_options(),
                       stream=torch.cuda.current_stream().cuda_stream)
    try:
        H.hdsw_factor(ctx)
        prob = O.Problem(w["kappa"], w["h"], w["W"])
        r = torch.from_numpy(np.stack([O.global_rhs(prob, fi) for fi in w["f"]])).cuda()
        rec = A.search(H, torch, ctx, r, 2, True, reps=3)
        assert H.hdsw_tuning_get(ctx) == rec["params"]
        assert rec["ms"] <= rec["default_ms"]
        assert len(rec["candidates"]) == len(A.candidates(2, True))
    finally:
        H.hdsw_destroy(ctx)
