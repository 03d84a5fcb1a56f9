"""Seeded synthetic inputs: wavenumber fields and point-like sources.

This module holds no arithmetic of the method.  It only produces the inputs
that both the HIP path and the FP64 oracle consume, so that both sides see
the same arrays.  Arrays use the reversed-axis layout of the library (x is
the last, fastest numpy axis), values on the N_x x N_y (x N_z) interior nodes
x_p = (p + 1/2) h of the box [0, N h]^d.

Workloads (the paper's own media and its BP-2004 model are not available;
these synthetic stand-ins have the shapes, sizes and wavenumber structure of
Sec. 5: constant media at a fixed number of points per wavelength, two-layer
media with a horizontal interface that avoids subdomain boundaries, and
Gaussian point-like sources at seeded positions):

  small2d : 128^2,  W 16, 2x2,   k = 16 pi,              1 RHS at (0.5, 0.5)
  c2d     : 1024^2, W 16, 8x8,   k = 2 pi / (10 h),     16 RHS, seed 20030260
  layer2d : 2048^2, W 16, 16x16, k1 = 2 pi/(10 h) below y = 0.37, 1.5 k1 above,
            64 RHS, seed 20030261, two rounds
  c3d     : 96^3,   W 6,  3x3x3, k = 2 pi / (8 h),       8 RHS, seed 20030262
"""

import numpy as np

SEED_BASE = 20030258


def node_coords(n, h):
    return (np.arange(n) + 0.5) * h


def constant_kappa(N, k):
    """Constant wavenumber on the interior nodes; N per axis (x first)."""
    return np.full(tuple(reversed(N)), float(k))


def two_layer_kappa(N, h, k_below, k_above, y_interface):
    """Two-layer wavenumber (eq. (2L-medium) with a horizontal interface):
    k_below where the node's y < y_interface, k_above elsewhere."""
    y = node_coords(N[1], h)
    layer = np.where(y < y_interface, float(k_below), float(k_above))
    shape = tuple(reversed(N))
    if len(N) == 2:
        return np.broadcast_to(layer[:, None], shape).copy()
    return np.broadcast_to(layer[None, :, None], shape).copy()


def gaussian_axis(n, h, c, sigma):
    """exp(-(x - c)^2 / (2 sigma^2)) on the n nodes of one axis."""
    x = node_coords(n, h)
    return np.exp(-(x - c) ** 2 / (2.0 * sigma * sigma))


def gaussian_mass(d, sigma):
    """(2 pi sigma^2)^{d/2}, the normalisation of a d-dimensional Gaussian."""
    return (2.0 * np.pi * sigma * sigma) ** (d / 2.0)


def gaussian_source(N, h, x0, sigma):
    """f(x) = exp(-|x - x0|^2 / (2 sigma^2)) / (2 pi sigma^2)^{d/2} on the
    interior nodes (a unit-mass smoothed point source), the product of the
    per-axis factors taken from x upwards."""
    d = len(N)
    out = np.ones(tuple(reversed(N)))
    for a in range(d):
        g = gaussian_axis(N[a], h, x0[a], sigma)
        shp = [1] * d
        shp[d - 1 - a] = N[a]
        out = out * g.reshape(shp)
    return out / gaussian_mass(d, sigma)


def random_positions(n, d, seed, lo, hi):
    """n seeded positions uniform in [lo, hi]^d."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, d))


def sources(N, h, positions, sigma):
    """Stack [nrhs][interior grid] of Gaussian sources (complex128)."""
    return np.stack([gaussian_source(N, h, p, sigma) for p in positions]
                    ).astype(np.complex128)


CONFIGS = {
    "small2d": dict(dim=2, N=128, W=16, P=2, ppw=None, k=16 * np.pi, nrhs=1,
                    rounds=1, layer=None, seed=None),
    "c2d": dict(dim=2, N=1024, W=16, P=8, ppw=10, k=None, nrhs=16, rounds=1,
                layer=None, seed=SEED_BASE + 2),
    "layer2d": dict(dim=2, N=2048, W=16, P=16, ppw=10, k=None, nrhs=64,
                    rounds=2, layer=(1.5, 0.37), seed=SEED_BASE + 3),
    "c3d": dict(dim=3, N=96, W=6, P=3, ppw=8, k=None, nrhs=8, rounds=1,
                layer=None, seed=SEED_BASE + 4),
}


def make(name, nrhs=None, **override):
    """Build (kappa, f[nrhs], h, W, P, rounds) for a named workload.  Keyword
    overrides (N, P, W, ppw, nrhs, ...) give scaled-down variants with the
    same recipe."""
    c = dict(CONFIGS[name])
    c.update(override)
    if nrhs is not None:
        c["nrhs"] = nrhs
    d, N = c["dim"], c["N"]
    h = 1.0 / N
    Ns = (N,) * d
    k = c["k"] if c["k"] is not None else 2 * np.pi / (c["ppw"] * h)
    if c["layer"] is None:
        kappa = constant_kappa(Ns, k)
    else:
        ratio, yi = c["layer"]
        kappa = two_layer_kappa(Ns, h, k, ratio * k, yi)
    if c["seed"] is None:
        pos = np.full((c["nrhs"], d), 0.5)
    else:
        pos = random_positions(c["nrhs"], d, c["seed"], 12 * h, 1 - 12 * h)
    f = sources(Ns, h, pos, 2 * h)
    return dict(kappa=kappa, f=f, h=h, W=c["W"], P=(c["P"],) * d,
                rounds=c["rounds"], positions=pos, k=k)


# ---------------------------------------------------------------- serving
# A request stream: Poisson arrivals of 2D solve requests whose operator key
# (grid size N, subdomain size n_a, medium, points per wavelength) comes from
# a small key space, so that factors are reused, each with R point sources.

SERVE_SIZES = (256, 512, 1024, 2048)
SERVE_SUBDOMAINS = (64, 128)
SERVE_PPW = (8, 10, 12)
SERVE_HEIGHTS = (0.37, 0.53, 0.71)
SERVE_RMAX = 32
SERVE_W = 16


def serve_kappa(key):
    """(kappa, h, P, W, rounds) of an operator key (N, n_a, y_interface, ppw);
    y_interface None is the constant medium, otherwise k2 = 1.5 k1 above it
    (one extra round of sweeps for the layered medium)."""
    N, n_a, yi, ppw = key
    h = 1.0 / N
    k = 2 * np.pi / (ppw * h)
    if yi is None:
        kap = constant_kappa((N, N), k)
    else:
        kap = two_layer_kappa((N, N), h, k, 1.5 * k, yi)
    return kap, h, (N // n_a, N // n_a), SERVE_W, (1 if yi is None else 2)


def request_stream(n, rate, seed=SEED_BASE + 5, sizes=SERVE_SIZES, subdomains=SERVE_SUBDOMAINS,
                   ppws=SERVE_PPW, heights=SERVE_HEIGHTS, rmax=SERVE_RMAX):
    """n requests as dicts (rid, arrival, key, positions [R][2]); arrival
    times are a Poisson process of the given rate (requests/s; None or inf:
    all at time 0).  Medium: constant with probability 1/2, else two-layer
    with a uniformly chosen interface height."""
    rng = np.random.default_rng(seed)
    if rate is None or not np.isfinite(rate):
        t = np.zeros(n)
    else:
        t = np.cumsum(rng.exponential(1.0 / rate, size=n))
        t -= t[0]
    out = []
    for i in range(n):
        N = int(rng.choice(sizes))
        n_a = int(rng.choice(subdomains))
        yi = None if rng.random() < 0.5 else float(rng.choice(heights))
        ppw = int(rng.choice(ppws))
        R = int(rng.integers(1, rmax + 1))
        h = 1.0 / N
        pos = rng.uniform(12 * h, 1 - 12 * h, size=(R, 2))
        out.append(dict(rid=i, arrival=float(t[i]), key=(N, n_a, yi, ppw), positions=pos))
    return out
