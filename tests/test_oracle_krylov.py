"""Pins of the oracle's refinement and GMRES drivers (Sec. 5.2: the DDM as
preconditioner of GMRES, stopped on the relative residual).  Both must reach
the global PML solution, the fixed point that the DDM only approximates, and
GMRES must take few iterations when the DDM is (nearly) exact: two rounds on
a two-layer medium (Thm 3.10) or one round on a constant medium (Thm 3.3).
With one round on a two-layer medium the DDM misses the waves the interface
sends back (Lemma 3.7: one round suffices only for sources below the
interface), and GMRES needs many more steps."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_2003_02585_amd import workloads as wl


def _setup(layer=None, N=64, P=(4, 4), pml_R=1e-16):
    h = 1.0 / N
    k = 2 * np.pi / (10 * h)
    kap = wl.constant_kappa((N, N), k) if layer is None else \
        wl.two_layer_kappa((N, N), h, k, layer * k, 0.37)
    prob = O.Problem(kap, h, 16, pml_R=pml_R)
    part = O.Partition(prob, P)
    sol = O.SubdomainSolvers(part)
    S = O.global_operator(prob)
    f = wl.gaussian_source((N, N), h, (0.31, 0.77), 2 * h) + \
        wl.gaussian_source((N, N), h, (0.6, 0.2), 2 * h)
    b = O.global_rhs(prob, f)
    return prob, part, sol, S, b


def _precond(prob, part, sol, rounds):
    def M(r):
        return O.ddm_apply(prob, part, r.reshape(prob.gshape), rounds=rounds,
                           solvers=sol).ravel()
    return M


def test_refinement_reaches_global_solution():
    prob, part, sol, S, b = _setup()
    ug = spla.splu(S.tocsc()).solve(b.ravel())
    x, hist = O.refine(S, b, _precond(prob, part, sol, 1), tol=1e-12, maxit=10)
    assert hist[-1] <= 1e-12 and len(hist) <= 5, hist
    # residual reduction per step is of the order of the DDM's layer error
    assert hist[1] < 1e-3
    assert np.linalg.norm(x - ug) / np.linalg.norm(ug) < 1e-10


def test_gmres_two_layer_matches_direct_solve():
    prob, part, sol, S, b = _setup(layer=1.5)
    ug = spla.splu(S.tocsc()).solve(b.ravel())
    for rounds, max_it in ((1, 12), (2, 4)):
        info = {}
        x, hist = O.gmres(S, b, _precond(prob, part, sol, rounds), m=20,
                          tol=1e-10, maxit=30, info=info)
        assert hist[-1] <= 1e-10, hist
        assert info["iters"] <= max_it, (rounds, info["iters"])
        assert np.linalg.norm(x - ug) / np.linalg.norm(ug) < 1e-8
    # GMRES on the unpreconditioned system is far slower (sanity of M)
    x0, h0 = O.gmres(S, b, lambda r: r, m=20, tol=1e-6, maxit=40)
    assert h0[-1] > 1e-6


def test_gmres_identity_preconditioner_small_dense():
    # GMRES itself against a dense solve on a tiny system
    prob, part, sol, S, b = _setup(N=16, P=(2, 2), pml_R=1e-4)
    x, hist = O.gmres(S, b, lambda r: r, m=30, tol=1e-12, maxit=2000)
    ref = np.linalg.solve(S.toarray(), b.ravel())
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10


@pytest.mark.slow
def test_one_round_gmres_two_layer_needs_long_krylov_spaces():
    # 256^2, 8 x 8 subdomains, k2 = 1.5 k1 above y = 0.37, a source above the
    # interface.  Two rounds (Thm 3.10): GMRES(20) converges in at most 4
    # steps.  One round: the preconditioned operator keeps the reflected
    # waves' part, GMRES needs tens of steps; unrestarted (m = 80) it reaches
    # 1e-10 within 60 steps, while restarts every 20 steps discard the
    # Krylov space and the iteration stalls above 1e-6 after 80 steps.
    N, P = 256, (8, 8)
    h = 1.0 / N
    k = 2 * np.pi / (10 * h)
    kap = wl.two_layer_kappa((N, N), h, k, 1.5 * k, 0.37)
    prob = O.Problem(kap, h, 16)
    part = O.Partition(prob, P)
    sol = O.SubdomainSolvers(part)
    S = O.global_operator(prob).tocsr()
    b = O.global_rhs(prob, wl.gaussian_source((N, N), h, (0.45, 0.77), 2 * h)).ravel()
    ug = spla.splu(S.tocsc()).solve(b)
    res = {}
    for rounds, m, maxit in ((2, 20, 20), (1, 80, 80), (1, 20, 80)):
        info = {}
        x, hist = O.gmres(S, b, _precond(prob, part, sol, rounds), m=m, tol=1e-10,
                          maxit=maxit, info=info)
        res[(rounds, m)] = (info["iters"], hist[-1], np.linalg.norm(x - ug) / np.linalg.norm(ug))
    it2, r2, e2 = res[(2, 20)]
    assert it2 <= 4 and r2 <= 1e-10 and e2 < 1e-8, res
    it1, r1, e1 = res[(1, 80)]
    assert 10 < it1 <= 60 and r1 <= 1e-10 and e1 < 1e-8, res
    it1r, r1r, _ = res[(1, 20)]
    assert it1r == 80 and r1r > 1e-6, res
