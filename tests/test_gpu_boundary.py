"""GPU tests of the C-ABI's contract around the method: allocator hooks,
argument checks on caller arrays, workspaces that grow between calls, and
results that do not depend on which other columns share a launch.

Every result is also held to the parity bars of the method (relative 2-norm
against the FP64 oracle's global solution, 1e-8 after iteration)."""

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


def _case(N, W, P, layer=None, nrhs=3, seed=11, ppw=10):
    h = 1.0 / N
    k = 2 * np.pi / (ppw * h)
    kap = wl.constant_kappa((N, N), k) if layer is None else \
        wl.two_layer_kappa((N, N), h, k, layer * k, 0.37)
    pos = wl.random_positions(nrhs, 2, seed, 4 * h, 1 - 4 * h)
    f = wl.sources((N, N), h, pos, 2 * h)
    prob = O.Problem(kap, h, W)
    b = np.stack([O.global_rhs(prob, fi) for fi in f])
    return dict(h=h, kap=kap, f=f, prob=prob, b=b, P=P, W=W)


def _ctx(H, c, **opt):
    stream = torch.cuda.current_stream().cuda_stream
    ctx = H.hdsw_setup(c["kap"], c["h"], c["P"], c["W"], H.hdsw_default_options(**opt),
                       stream=stream)
    H.hdsw_factor(ctx)
    return ctx


def _rel(a, b):
    return max(np.linalg.norm(x - y) / np.linalg.norm(y) for x, y in zip(a, b))


def test_allocator_hooks_own_every_allocation(H):
    # every device allocation goes through the caller's hooks (here torch's
    # caching allocator); the results equal those of a context that uses
    # hipMalloc, bit for bit, and destroy hands every block back
    c = _case(64, 16, (4, 4), 1.5, nrhs=3)
    _say("allocator hooks")
    alloc, free, live = H.torch_allocator_hooks()
    ft = torch.from_numpy(c["f"]).cuda()
    out = []
    for hooks in (dict(dev_alloc=alloc, dev_free=free), {}):
        ctx = _ctx(H, c, precision=H.HDSW_MIXED, rounds=2, tol=1e-10, **hooks)
        try:
            if hooks:
                fb, _, ws = H.hdsw_query(ctx)
                held = sum(t.numel() for t in live.values())
                assert held >= fb and len(live) > 5
            xt = torch.zeros_like(ft)
            H.hdsw_solve(ctx, ft, xt, 3)
            out.append(xt.cpu().numpy())
        finally:
            H.hdsw_destroy(ctx)
        if hooks:
            assert not live, f"{len(live)} blocks not returned"
    assert np.array_equal(out[0], out[1])
    ug = O.solve_global(c["prob"], c["b"])
    sl = c["prob"].interior_slice()
    assert _rel(out[0], [u[sl] for u in ug]) < 1e-8


def test_allocator_hook_failure_is_enomem(H):
    # a hook that returns NULL makes setup fail with ENOMEM, after handing
    # back what it had taken
    c = _case(32, 8, (2, 2), nrhs=1)
    _say("allocator hook failure")
    alloc, free, live = H.torch_allocator_hooks()
    calls = [0]

    def _limited(nbytes, ctxp):
        calls[0] += 1
        return alloc(nbytes, ctxp) if calls[0] <= 3 else None

    lim = H.DEV_ALLOC_FN(_limited)
    opt = H.hdsw_default_options(dev_alloc=lim, dev_free=free)
    with pytest.raises(H.HdswError) as ei:
        H.hdsw_setup(c["kap"], c["h"], c["P"], c["W"], opt,
                     stream=torch.cuda.current_stream().cuda_stream)
    assert ei.value.status == H.HDSW_ENOMEM
    assert not live
    # one hook without the other is an argument error
    with pytest.raises(H.HdswError) as ei:
        H.hdsw_setup(c["kap"], c["h"], c["P"], c["W"], H.hdsw_default_options(dev_alloc=alloc))
    assert ei.value.status == H.HDSW_EINVAL


def test_host_pointers_are_rejected_before_any_launch(H):
    # pinned host memory is readable by the device, so a missing check would
    # not fault; the library must refuse it with EINVAL and stay usable
    c = _case(48, 8, (3, 3), nrhs=2)
    _say("host pointer checks")
    ctx = _ctx(H, c, precision=H.HDSW_MIXED, tol=1e-10)
    try:
        fh = torch.from_numpy(c["f"]).pin_memory()
        bh = torch.from_numpy(c["b"]).pin_memory()
        fd = fh.cuda()
        bd = bh.cuda()
        xd = torch.zeros_like(fd)
        zd = torch.zeros_like(bd)
        lib = H._lib
        import ctypes
        P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        assert lib.hdsw_solve(ctx, P(fh), P(xd), 2, None) == H.HDSW_EINVAL
        assert lib.hdsw_solve(ctx, P(fd), P(fh), 2, None) == H.HDSW_EINVAL
        assert lib.hdsw_apply_precond(ctx, P(bh), P(zd), 2) == H.HDSW_EINVAL
        assert lib.hdsw_residual(ctx, P(bd), P(bh), P(zd), 2, None) == H.HDSW_EINVAL
        # the binding refuses host tensors and arrays shorter than nrhs columns
        with pytest.raises(TypeError):
            H.hdsw_solve(ctx, fh, xd, 2)
        with pytest.raises(ValueError):
            H.hdsw_solve(ctx, fd[:1].contiguous(), xd, 2)
        with pytest.raises(ValueError):
            H.hdsw_apply_precond(ctx, bd, zd[:1].contiguous(), 2)
        # still usable
        info, _ = H.hdsw_solve(ctx, fd, xd, 2)
        x = xd.cpu().numpy()
    finally:
        H.hdsw_destroy(ctx)
    ug = O.solve_global(c["prob"], c["b"])
    sl = c["prob"].interior_slice()
    assert _rel(x, [u[sl] for u in ug]) < 1e-8


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_gmres_workspace_regrows(H, prec):
    # one GMRES context solves 1 column, then 3: the Krylov basis must grow
    # with the workspaces; both solves against the oracle's global solution
    c = _case(64, 16, (4, 4), 1.5, nrhs=3, seed=31)
    ug = O.solve_global(c["prob"], c["b"])
    sl = c["prob"].interior_slice()
    _say(f"gmres regrow {prec}")
    p = H.HDSW_FP64 if prec == "fp64" else H.HDSW_MIXED
    ctx = _ctx(H, c, precision=p, rounds=2, gmres_m=20, tol=1e-11, max_iter=40)
    try:
        ft = torch.from_numpy(c["f"]).cuda()
        x1 = torch.zeros_like(ft[:1])
        H.hdsw_solve(ctx, ft[:1].contiguous(), x1, 1)
        x3 = torch.zeros_like(ft)
        info, _ = H.hdsw_solve(ctx, ft, x3, 3)
        x1, x3 = x1.cpu().numpy(), x3.cpu().numpy()
    finally:
        H.hdsw_destroy(ctx)
    e1 = _rel(x1, [ug[0][sl]])
    e3 = _rel(x3, [u[sl] for u in ug])
    _say(f"  rel err 1 column {e1:.3e}, 3 columns {e3:.3e}, iterations {info}")
    assert e1 < 1e-8 and e3 < 1e-8


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_gmres_is_batch_invariant(H, prec):
    # a GMRES column takes its update from its own Arnoldi steps only, so it
    # is the same alone and inside a batch whose other columns need more
    # steps (one round on a two-layer medium: sources below the interface
    # converge in fewer iterations than those above it)
    c = _case(64, 16, (4, 4), 1.5, nrhs=3, seed=37)
    f = c["f"]
    _say(f"gmres batch invariance {prec}")
    p = H.HDSW_FP64 if prec == "fp64" else H.HDSW_MIXED
    ctx = _ctx(H, c, precision=p, rounds=1, gmres_m=20, tol=1e-10, max_iter=60)
    try:
        ft = torch.from_numpy(f).cuda()
        xb = torch.zeros_like(ft)
        info, _ = H.hdsw_solve(ctx, ft, xb, 3)
        alone, ia = [], []
        for j in range(3):
            xj = torch.zeros_like(ft[j:j + 1])
            i1, _ = H.hdsw_solve(ctx, ft[j:j + 1].contiguous(), xj, 1)
            alone.append(xj.cpu().numpy()[0])
            ia.append(i1[0][0])
        xb = xb.cpu().numpy()
    finally:
        H.hdsw_destroy(ctx)
    _say(f"  iterations batch {[i for i, _ in info]} alone {ia}")
    assert [i for i, _ in info] == ia
    for j in range(3):
        assert np.array_equal(xb[j], alone[j])


def test_sweep_step_split_does_not_depend_on_columns(H):
    # 2048^2 with 128^2 subdomains (a serving key): its large sweep steps take
    # the four-tile form.  One column alone and the same column among 20
    # columns (where a column-count rule would have switched forms) agree
    # bit for bit
    N, P = 2048, (16, 16)
    h = 1.0 / N
    k = 2 * np.pi / (10 * h)
    kap = wl.constant_kappa((N, N), k)
    pos = wl.random_positions(20, 2, 41, 12 * h, 1 - 12 * h)
    f = wl.sources((N, N), h, pos, 2 * h)
    _say("sweep-step form vs column count (2048^2, 16x16, 20 columns)")
    c = dict(kap=kap, h=h, P=P, W=16)
    ctx = _ctx(H, c, precision=H.HDSW_MIXED, tol=1e-10)
    try:
        ft = torch.from_numpy(f).cuda()
        xb = torch.zeros_like(ft)
        info, _ = H.hdsw_solve(ctx, ft, xb, 20)
        xa = torch.zeros_like(ft[:1])
        ia, _ = H.hdsw_solve(ctx, ft[3:4].contiguous(), xa, 1)
        same = bool(torch.equal(xb[3], xa[0]))
    finally:
        H.hdsw_destroy(ctx)
    _say(f"  iterations {info[3][0]} / {ia[0][0]}, equal {same}")
    assert info[3][0] == ia[0][0]
    assert same
