"""Pins of the oracle's discretization and direct solvers against what the
mathematics fixes independently of the oracle's own code: closed forms of
the Dirichlet Laplacian (DST), sine-mode eigenpairs, library dense solves,
complex symmetry / reciprocity, and the free-space Hankel solution."""

import numpy as np
import pytest
import scipy.fft
import scipy.special

import oracle as O
from paper_2003_02585_amd import workloads as wl


def _problem(N, W, k, dim=2, s0=None, layer=None):
    h = 1.0 / N
    Ns = (N,) * dim
    if layer is None:
        kap = wl.constant_kappa(Ns, k)
    else:
        kap = wl.two_layer_kappa(Ns, h, k, layer * k, 0.37)
    return O.Problem(kap, h, W, sigma0=s0)


@pytest.mark.parametrize("dim", [2, 3])
def test_operator_complex_symmetric(dim):
    # Discrete counterpart of the adjoint relation eq. (fund_sol_sym): the
    # J-scaled operator is complex symmetric, bit for bit.
    N, W = (24, 6) if dim == 2 else (8, 3)
    prob = _problem(N, W, 2 * np.pi / (8.0 / N), dim=dim, layer=1.5)
    S = O.global_operator(prob)
    assert (S != S.T).nnz == 0
    part = O.Partition(prob, (2,) * dim)
    for i in part.subdomains():
        Si = part.operator(i)
        assert (Si != Si.T).nnz == 0


def _dirichlet_eigs(M):
    k = np.arange(1, M + 1)
    return -4.0 * np.sin(np.pi * k / (2.0 * (M + 1))) ** 2


@pytest.mark.parametrize("dim", [2, 3])
def test_laplacian_closed_form_dst(dim):
    # sigma0 = 0, kappa = 0: S is the Dirichlet 5-/7-point Laplacian, which
    # the orthonormal type-I DST diagonalizes.
    N, W = (20, 4) if dim == 2 else (6, 2)
    prob = O.Problem(np.zeros((N,) * dim), 1.0 / N, W, sigma0=0.0)
    M = N + 2 * W
    rng = np.random.default_rng(1)
    b = rng.standard_normal((M,) * dim) + 1j * rng.standard_normal((M,) * dim)
    u = O.solve_global(prob, b, method="banded")
    lam = np.zeros((M,) * dim)
    for a in range(dim):
        shp = [1] * dim
        shp[a] = M
        lam = lam + _dirichlet_eigs(M).reshape(shp)
    bh = scipy.fft.dstn(b, type=1, norm="ortho")
    ref = scipy.fft.idstn(bh / lam, type=1, norm="ortho")
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-12


def test_sine_modes_are_eigenvectors():
    # sigma0 = 0, constant kappa: S v = (h^2 k^2 - sum 4 sin^2) v for every
    # separable sine mode.
    N, W = 16, 4
    h = 1.0 / N
    k = 9.0
    prob = O.Problem(np.full((N, N), k), h, W, sigma0=0.0)
    S = O.global_operator(prob)
    M = N + 2 * W
    p = np.arange(M)
    for (kx, ky) in [(1, 1), (3, 7), (M, 2), (5, M - 1)]:
        v = np.outer(np.sin(np.pi * ky * (p + 1) / (M + 1)),
                     np.sin(np.pi * kx * (p + 1) / (M + 1)))
        lam = h * h * k * k - 4 * np.sin(np.pi * kx / (2 * (M + 1))) ** 2 \
            - 4 * np.sin(np.pi * ky / (2 * (M + 1))) ** 2
        Sv = (S @ v.ravel()).reshape(v.shape)
        assert np.abs(Sv - lam * v).max() < 1e-13 * max(1.0, abs(lam))


@pytest.mark.parametrize("dim", [2, 3])
def test_banded_solve_matches_dense(dim):
    N, W = (8, 4) if dim == 2 else (4, 2)
    prob = _problem(N, W, 2 * np.pi / (6.0 / N), dim=dim, layer=1.5)
    S = O.global_operator(prob)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(prob.gshape) + 1j * rng.standard_normal(prob.gshape)
    u = O.solve_global(prob, b, method="banded")
    ref = np.linalg.solve(S.toarray(), b.ravel()).reshape(b.shape)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-12
    # subdomain factors too
    part = O.Partition(prob, (2,) * dim)
    sol = O.SubdomainSolvers(part)
    for i in part.subdomains():
        r = rng.standard_normal(part.ext_shape()) + 0j
        x = sol.solve(i, r)
        xr = np.linalg.solve(sol.ops[i].toarray(), r.ravel()).reshape(r.shape)
        assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-12


def test_reciprocity():
    # (S^-1)_{ab} = (S^-1)_{ba}: symmetric Green's function.
    prob = _problem(16, 6, 2 * np.pi / (8.0 / 16), layer=1.5)
    n = int(np.prod(prob.gshape))
    rng = np.random.default_rng(3)
    a, b = rng.choice(n, size=2, replace=False)
    ea = np.zeros(n, complex)
    ea[a] = 1
    eb = np.zeros(n, complex)
    eb[b] = 1
    ua = O.solve_global(prob, ea.reshape(prob.gshape)).ravel()
    ub = O.solve_global(prob, eb.reshape(prob.gshape)).ravel()
    assert abs(ua[b] - ub[a]) <= 1e-12 * abs(ua[b])


def test_free_space_hankel_second_order():
    # The global PML solution for a unit-mass Gaussian source converges at
    # second order to the radiating solution of eq. (helm)-(radiation),
    # u = -(i/4) exp(-k^2 s^2 / 2) H0^(1)(k r) away from the source (the
    # paper's L G = -delta convention).  This pins the operator's sign, its
    # J / A scaling and the absorbing layer at once.
    k = 8 * np.pi
    sig = 1.0 / 32
    errs = []
    for N in (64, 128, 256):
        h = 1.0 / N
        W = N // 8                       # fixed physical layer depth 1/8
        prob = O.Problem(np.full((N, N), k), h, W)
        f = wl.gaussian_source((N, N), h, (0.5, 0.5), sig)
        u = O.solve_global(prob, O.global_rhs(prob, f), method="sparse")
        x = (np.arange(N) + 0.5) * h
        X, Y = np.meshgrid(x, x)
        r = np.hypot(X - 0.5, Y - 0.5)
        mask = (r > 0.2) & (r < 0.42)
        ui = u[prob.interior_slice()]
        ref = -0.25j * np.exp(-0.5 * (k * sig) ** 2) * scipy.special.hankel1(0, k * r)
        errs.append(np.linalg.norm((ui - ref)[mask]) / np.linalg.norm(ref[mask]))
    assert errs[-1] < 2e-2
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


def test_discrete_dispersion_phase_slope():
    # Plane-wave consistency: along a grid axis, away from source and layer,
    # the phase of the discrete solution advances at the discrete wavenumber
    # (2/h) asin(k h / 2) of the 1D three-point stencil.
    N, W = 256, 32
    h = 1.0 / N
    k = 2 * np.pi / (16 * h)
    prob = O.Problem(np.full((N, N), k), h, W)
    f = wl.gaussian_source((N, N), h, (0.5, 0.5), 2 * h)
    u = O.solve_global(prob, O.global_rhs(prob, f), method="sparse")
    ui = u[prob.interior_slice()]
    row = ui[N // 2 - 1] + ui[N // 2]          # symmetric about y = 0.5
    xs = np.arange(N // 2 + 40, N - 24)
    ph = np.unwrap(np.angle(row[xs]))
    # outgoing cylindrical wave: phase = k_d r + const, amplitude ~ r^-1/2
    slope = np.polyfit(xs * h, ph, 1)[0]
    kd = 2.0 / h * np.arcsin(k * h / 2)
    assert abs(slope - kd) / kd < 3e-3, (slope, kd, k)
