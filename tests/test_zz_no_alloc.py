"""GPU test of hdsw_apply_precond_noalloc, the allocation-free DDM
application: through the C-ABI, against hdsw_apply_precond on the same
context (same kernels, so bit for bit) and against the FP64 oracle's
Algorithm 2.1 / 4.1 (1e-10), on two calls in a row, the second with fewer
columns, so that what the first call left in the shared array cannot reach
the second one's results."""

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
    stream = torch.cuda.current_stream().cuda_stream
    ctx = H.hdsw_setup(kap, h, P, W, H.hdsw_default_options(**opt), stream=stream)
    H.hdsw_factor(ctx)
    return ctx


def _two_calls(H, ctx, b, small):
    """Reference (allocating entry point) and allocation-free results for all
    columns of b, then for the first `small` columns."""
    r = torch.from_numpy(b).cuda()
    ref = torch.zeros_like(r)
    H.hdsw_apply_precond(ctx, r, ref, r.shape[0])
    z1 = torch.full_like(r, 3.0)
    H.hdsw_apply_precond_noalloc(ctx, r, z1, r.shape[0])
    rs = r[:small].contiguous()
    z2 = torch.full_like(rs, -5.0)
    H.hdsw_apply_precond_noalloc(ctx, rs, z2, small)
    return ref.cpu().numpy(), z1.cpu().numpy(), z2.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_2d(H, prec):
    N, W, P = 48, 8, (3, 3)
    h = 1.0 / N
    kap = wl.two_layer_kappa((N, N), h, 2 * np.pi / (10 * h), 3 * np.pi / (10 * h), 0.37)
    f = wl.sources((N, N), h, wl.random_positions(3, 2, 7, 4 * h, 1 - 4 * h), 2 * h)
    prob = O.Problem(kap, h, W)
    part = O.Partition(prob, P)
    b = np.stack([O.global_rhs(prob, fi) for fi in f])
    sol = O.SubdomainSolvers(part)
    oref = [O.ddm_apply(prob, part, bi, rounds=2, solvers=sol) for bi in b]
    _say(f"noalloc 2d {prec}")
    p = H.HDSW_FP64 if prec == "fp64" else H.HDSW_MIXED
    ctx = _ctx(H, kap, h, P, W, precision=p, rounds=2)
    try:
        ref, z1, z2 = _two_calls(H, ctx, b, 1)
    finally:
        H.hdsw_destroy(ctx)
    assert np.array_equal(z1, ref)
    assert np.array_equal(z2[0], ref[0])
    e = max(np.linalg.norm(z - o) / np.linalg.norm(o) for z, o in zip(z1, oref))
    _say(f"  rel diff vs oracle {e:.3e}")
    assert e < (1e-10 if prec == "fp64" else 2e-4)


def test_noalloc_3d(H):
    Ns, W, P = (12, 12, 12), 3, (2, 2, 2)
    h = 1.0 / Ns[0]
    kap = wl.constant_kappa(Ns, 2 * np.pi / (6 * h))
    f = wl.sources(Ns, h, wl.random_positions(2, 3, 7, 0.2, 0.8), 2 * h)
    prob = O.Problem(kap, h, W, pml_R=1e-4)
    part = O.Partition(prob, P)
    b = np.stack([O.global_rhs(prob, fi) for fi in f])
    oref = [O.ddm_apply(prob, part, bi) for bi in b]
    _say("noalloc 3d fp64")
    ctx = _ctx(H, kap, h, P, W, precision=H.HDSW_FP64, pml_R=1e-4)
    try:
        ref, z1, z2 = _two_calls(H, ctx, b, 1)
    finally:
        H.hdsw_destroy(ctx)
    assert np.array_equal(z1, ref)
    assert np.array_equal(z2[0], ref[0])
    e = max(np.linalg.norm(z - o) / np.linalg.norm(o) for z, o in zip(z1, oref))
    _say(f"  rel diff vs oracle {e:.3e}")
    assert e < 1e-10


def test_noalloc_in_passes_at_full_size(H):
    # 1024^2, 8 x 8, complex64: about 17 MB of workspace per column, so 8
    # columns run in passes of 3 through the 64 MiB array; then 2 columns
    w = wl.make("c2d", nrhs=8)
    prob = O.Problem(w["kappa"], w["h"], w["W"])
    b = np.stack([O.global_rhs(prob, fi) for fi in w["f"]])
    _say("noalloc c2d 8 columns in passes")
    ctx = _ctx(H, w["kappa"], w["h"], w["P"], w["W"], precision=H.HDSW_MIXED)
    try:
        ref, z1, z2 = _two_calls(H, ctx, b, 2)
    finally:
        H.hdsw_destroy(ctx)
    assert np.array_equal(z1, ref)
    assert np.array_equal(z2, ref[:2])


def test_noalloc_refuses_columns_beyond_the_array(H):
    # 2048^2, 16 x 16, two rounds: one column needs about 74 MB > 64 MiB
    w = wl.make("layer2d", nrhs=1)
    prob = O.Problem(w["kappa"], w["h"], w["W"])
    b = O.global_rhs(prob, w["f"][0])[None]
    _say("noalloc refusal (2048^2, 16x16, two rounds)")
    ctx = _ctx(H, w["kappa"], w["h"], w["P"], w["W"], precision=H.HDSW_MIXED, rounds=2)
    try:
        r = torch.from_numpy(b).cuda()
        z = torch.zeros_like(r)
        with pytest.raises(H.HdswError) as ei:
            H.hdsw_apply_precond_noalloc(ctx, r, z, 1)
        assert ei.value.status == H.HDSW_ENOMEM
        # the context is still usable
        H.hdsw_apply_precond(ctx, r, z, 1)
        assert torch.isfinite(torch.view_as_real(z)).all()
    finally:
        H.hdsw_destroy(ctx)
