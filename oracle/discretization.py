"""Grid, PML and finite-difference operator of the oracle.

Conventions (fixed here, restated in the test fixtures):

* Interior box B = prod_a [0, N_a h].  Nodes are cell-centred,
  x_p = (p + 1/2) h, global node indices p = -W .. N_a + W - 1 per axis, so a
  subdomain interface (a multiple of h) always falls on a half-point and no
  node carries the value 1/2 of the discontinuous cutoff (Sec. 2.2, mu).
* Homogeneous Dirichlet data at the ghost nodes p = -W - 1 and p = N_a + W
  truncate the layer (the paper poses the PML on all of R^n, eq. (PML)).
* Grid arrays are numpy arrays whose shape is the per-axis node counts in
  REVERSED order, so axis 0 (x) is the last, fastest numpy axis.

PML (Sec. 2.1, eq. (sigma) and the stretching after it): sigma_j is a profile
of the distance t outside the box; the paper leaves the profile open, the
oracle takes sigma(t) = sigma0 (t/delta)^2 with delta = W h and
alpha_j = 1 + i sigma_j.  One sigma0 serves the global problem and every
subdomain.

Operator (eq. (PML) in 2D, eq. (PML3) in 3D, multiplied by h^2 J): with
a^a at the half-point between nodes p and p+1 along axis a equal to
prod_{b != a} alpha_b(x_b) / alpha_a(x_{p+1/2}),

  (S u)_p = sum_a [ a^a_{p+1/2}(u_{p+e_a} - u_p) - a^a_{p-1/2}(u_p - u_{p-e_a}) ]
            + h^2 kappa_p^2 J_p u_p ,   J = prod_a alpha_a,

and the right-hand side is b = h^2 J f.  S is complex symmetric, the discrete
counterpart of the adjoint relation eq. (fund_sol_sym) for the J-scaled form.
"""

import numpy as np
import scipy.sparse as sp


def sigma0_from_R(pml_R, kappa_ref, W, h):
    """sigma0 giving a nominal layer attenuation pml_R for the quadratic
    profile: 3 ln(1/R) / (kappa_ref * W h).  (The paper leaves the profile
    open, Sec. 2.1; this choice is the oracle's reading.)"""
    delta = W * h
    return 3.0 * np.log(1.0 / pml_R) / (kappa_ref * delta)


def alpha(x, lo, hi, s0, delta):
    """alpha(x) = 1 + i sigma(t(x)), t = distance of x outside [lo, hi]
    (Sec. 2.1, eq. (sigma) with the quadratic profile)."""
    x = np.asarray(x, dtype=float)
    t = np.maximum(0.0, np.maximum(lo - x, x - hi))
    return 1.0 + 1j * (s0 * (t / delta) ** 2)


def _bshape(dim, a, n):
    """Shape that puts a length-n vector on the numpy axis of grid axis a."""
    s = [1] * dim
    s[dim - 1 - a] = n
    return tuple(s)


def assemble(p0, p1, lo, hi, kappa, h, s0, W):
    """Sparse S on the nodes p0[a] <= p < p1[a] of each axis a, with Dirichlet
    ghosts at p0[a]-1 and p1[a], PML measured from the box [lo[a], hi[a]].

    kappa: real array on these nodes (reversed-axis shape).  Returns a CSR
    matrix in the flat C order of that array (x fastest)."""
    dim = len(p0)
    n = [p1[a] - p0[a] for a in range(dim)]
    shape = tuple(reversed(n))
    kappa = np.asarray(kappa, dtype=float)
    assert kappa.shape == shape, (kappa.shape, shape)
    delta = W * h
    # alpha at nodes and at the half-points p*h (between nodes p-1 and p),
    # for p = p0 .. p1 (n+1 half-points including the two ghost faces).
    al_node = [alpha((np.arange(p0[a], p1[a]) + 0.5) * h, lo[a], hi[a], s0, delta)
               .reshape(_bshape(dim, a, n[a])) for a in range(dim)]
    al_half = [alpha(np.arange(p0[a], p1[a] + 1) * h, lo[a], hi[a], s0, delta)
               .reshape(_bshape(dim, a, n[a] + 1)) for a in range(dim)]
    J = np.ones(shape, dtype=complex)
    for a in range(dim):
        J = J * al_node[a]
    diag = (h * h) * kappa ** 2 * J
    idx = np.arange(int(np.prod(n))).reshape(shape)
    rows, cols, vals = [], [], []
    for a in range(dim):
        ax = dim - 1 - a
        tang = np.ones((1,) * dim, dtype=complex)
        for b in range(dim):
            if b != a:
                tang = tang * al_node[b]
        coef = tang / al_half[a]                       # n[a]+1 faces along ax
        coef = np.broadcast_to(coef, tuple(
            (n[a] + 1) if k == ax else shape[k] for k in range(dim)))
        lower = np.take(coef, np.arange(0, n[a]), axis=ax)     # face p-1/2
        upper = np.take(coef, np.arange(1, n[a] + 1), axis=ax)  # face p+1/2
        diag = diag - lower - upper
        inner = np.take(coef, np.arange(1, n[a]), axis=ax)     # faces between nodes
        lo_idx = np.take(idx, np.arange(0, n[a] - 1), axis=ax)
        hi_idx = np.take(idx, np.arange(1, n[a]), axis=ax)
        rows += [lo_idx.ravel(), hi_idx.ravel()]
        cols += [hi_idx.ravel(), lo_idx.ravel()]
        vals += [inner.ravel(), inner.ravel()]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    N = int(np.prod(n))
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                                              np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    S.sort_indices()
    return S


class Problem:
    """The global PML problem P_{B,kappa} (Sec. 2.1) on the cell-centred grid.

    kappa: real wavenumber on the interior nodes of B (reversed-axis shape).
    In the layer the wavenumber is that of the nearest interior node (index
    clamping), the same nearest-point rule as eq. (wave_number)."""

    def __init__(self, kappa, h, W, pml_R=1e-16, sigma0=None):
        self.kappa = np.asarray(kappa, dtype=float)
        self.dim = self.kappa.ndim
        self.N = tuple(reversed(self.kappa.shape))
        self.h = float(h)
        self.W = int(W)
        self.s0 = float(sigma0) if sigma0 is not None else \
            sigma0_from_R(pml_R, float(self.kappa.min()), self.W, self.h)

    @property
    def M(self):
        return tuple(n + 2 * self.W for n in self.N)

    @property
    def gshape(self):
        """Reversed-axis shape of the global grid (interior plus layer)."""
        return tuple(reversed(self.M))

    def kappa_on(self, p0, p1, q0, q1):
        """kappa on nodes [p0, p1) per axis, each index clamped into
        [q0, q1 - 1] (the nearest-point extension, eq. (wave_number))."""
        dim = self.dim
        idx = []
        for a in range(dim):
            p = np.clip(np.arange(p0[a], p1[a]), q0[a], q1[a] - 1)
            idx.append(p)
        # numpy axes are reversed: build an open mesh in reversed order
        mesh = np.ix_(*[idx[a] for a in reversed(range(dim))])
        return self.kappa[mesh]

    def interior_slice(self):
        """Slice of the global grid array that holds the interior of B."""
        W = self.W
        return tuple(slice(W, W + n) for n in reversed(self.N))


def global_operator(prob):
    """S for P_{B,kappa} on the whole global grid."""
    dim, W, h = prob.dim, prob.W, prob.h
    p0 = [-W] * dim
    p1 = [prob.N[a] + W for a in range(dim)]
    lo = [0.0] * dim
    hi = [prob.N[a] * h for a in range(dim)]
    kap = prob.kappa_on(p0, p1, [0] * dim, list(prob.N))
    return assemble(p0, p1, lo, hi, kap, h, prob.s0, W)


def global_rhs(prob, f):
    """b = h^2 J f on the global grid; f is given on the interior nodes of B
    and is zero in the layer (f is supported in B, Sec. 2.1)."""
    dim, h = prob.dim, prob.h
    f = np.asarray(f)
    b = np.zeros(prob.gshape, dtype=complex)
    sl = prob.interior_slice()
    # J on interior nodes: alpha = 1 + i sigma(0) for every axis
    J = np.ones(f.shape, dtype=complex)
    for a in range(dim):
        x = (np.arange(prob.N[a]) + 0.5) * h
        al = alpha(x, 0.0, prob.N[a] * h, prob.s0, prob.W * h)
        J = J * al.reshape(_bshape(dim, a, prob.N[a]))
    b[sl] = (h * h) * J * f
    return b


class Partition:
    """Checkerboard partition of B into prod_a P_a boxes (Sec. 2.3 in 2D,
    Sec. 4 in 3D); subdomain index i = (i_0, .., i_{d-1}), 0-based.

    Subdomain i has interior nodes [i_a n_a, (i_a+1) n_a) per axis, its own
    layer of W nodes on every side measured from its own box, the same
    sigma0, and the wavenumber extended by the nearest interior node of the
    subdomain (eq. (wave_number)).  Ownership (the cutoff mu_{i,j} with its
    "1 otherwise" case on outer sides) adds the global-layer nodes beyond the
    outer faces of boundary subdomains."""

    def __init__(self, prob, P):
        self.prob = prob
        self.dim = prob.dim
        self.P = tuple(int(p) for p in P)
        assert len(self.P) == self.dim
        for a in range(self.dim):
            assert prob.N[a] % self.P[a] == 0, "N must be divisible by P"
        self.n = tuple(prob.N[a] // self.P[a] for a in range(self.dim))
        self.W = prob.W

    def subdomains(self):
        return [tuple(int(v) for v in reversed(t)) for t in
                np.ndindex(*tuple(reversed(self.P)))]

    def ext_range(self, i):
        W = self.W
        p0 = [i[a] * self.n[a] - W for a in range(self.dim)]
        p1 = [(i[a] + 1) * self.n[a] + W for a in range(self.dim)]
        return p0, p1

    def ext_shape(self):
        return tuple(reversed([n + 2 * self.W for n in self.n]))

    def box(self, i):
        h = self.prob.h
        lo = [i[a] * self.n[a] * h for a in range(self.dim)]
        hi = [(i[a] + 1) * self.n[a] * h for a in range(self.dim)]
        return lo, hi

    def kappa_sub(self, i):
        p0, p1 = self.ext_range(i)
        q0 = [i[a] * self.n[a] for a in range(self.dim)]
        q1 = [(i[a] + 1) * self.n[a] for a in range(self.dim)]
        return self.prob.kappa_on(p0, p1, q0, q1)

    def operator(self, i):
        p0, p1 = self.ext_range(i)
        lo, hi = self.box(i)
        return assemble(p0, p1, lo, hi, self.kappa_sub(i), self.prob.h,
                        self.prob.s0, self.W)

    def owned_range(self, i):
        """Owned global node range per axis (mu_{i,j}, including the
        global-layer nodes beyond outer faces)."""
        W, N = self.W, self.prob.N
        o0 = [i[a] * self.n[a] if i[a] > 0 else -W for a in range(self.dim)]
        o1 = [(i[a] + 1) * self.n[a] if i[a] < self.P[a] - 1 else N[a] + W
              for a in range(self.dim)]
        return o0, o1

    def owned_slices(self, i):
        """(slice into the global array, slice into the subdomain array)."""
        W = self.W
        p0, _ = self.ext_range(i)
        o0, o1 = self.owned_range(i)
        g = tuple(slice(o0[a] + W, o1[a] + W) for a in reversed(range(self.dim)))
        l = tuple(slice(o0[a] - p0[a], o1[a] - p0[a])
                  for a in reversed(range(self.dim)))
        return g, l
