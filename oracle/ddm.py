"""Algorithm 2.1 (2D) and Algorithm 4.1 (3D), step by step, in FP64.

Discrete trace transfer (Lemma 2.2 and the remark that closes Sec. 2.3: the
potentials are realised as subdomain solves with particular sources that are
summed into one right-hand side):

* The transferred trace a subdomain sends across the interface between
  global node layers m and m+1 of axis a is the pair (v[m], v[m+1]) of its
  own solution v on the two layers next to the interface, over the whole
  tangential extent of its extended grid.  For the sender one layer is its
  last interior layer and the other its first layer inside its own PML.
* The receiver turns the pair into the source g = [S_r, chi_r] v~, where v~
  is the pair placed on the receiver's grid, S_r the receiver's operator and
  chi_r the indicator of the receiver's half-space.  For the global operator
  and v = u this source reproduces u chi_R exactly (u chi_R = S^{-1} [S,chi_R] u
  when b vanishes on R), the discrete statement of eq. (trace_potential_total).
  This commutator form has no normal-sign convention to choose.

Everything else follows Algorithm 2.1 / 4.1: sweep list, step groups, solve
with the subdomain source only the first time a subdomain is visited (then
f_ij = 0), skip the solve when the whole right-hand side is exactly zero,
route each of the 2n traces to the smallest admissible sweep, and sum the
local solutions on owned nodes (u_DDM = sum_l sum_ij u^l_ij mu_ij).
"""

import hashlib

import numpy as np

from .banded import BandedLU, band_of
from .routing import sweep_directions, step_groups, route


class SubdomainSolvers:
    """Subdomain operators S_ij with banded LU factors; identical operators
    (byte-identical CSR data) share one factor when dedup is on."""

    def __init__(self, part, dedup=True):
        self.part = part
        self.ops = {}
        self.key = {}
        self.factors = {}
        kb = band_of(part.ext_shape())
        for i in part.subdomains():
            S = part.operator(i)
            k = hashlib.sha256(S.data.tobytes() + S.indices.tobytes() +
                               S.indptr.tobytes()).hexdigest() if dedup else i
            self.ops[i] = S
            self.key[i] = k
            if k not in self.factors:
                self.factors[k] = BandedLU(S, kb)

    @property
    def n_distinct(self):
        return len(self.factors)

    def solve(self, i, rhs):
        shp = rhs.shape
        return self.factors[self.key[i]].solve(rhs.ravel()).reshape(shp)


def _layers(part, a, side):
    """Local layer indices (m, m+1) along axis a of the interface on the
    given side (-1 lower, +1 upper) of a subdomain's extended grid."""
    W, n = part.W, part.n[a]
    if side < 0:
        return W - 1, W
    return W + n - 1, W + n


def extract_trace(part, v, a, side, incoming=None):
    """Trace sent across this subdomain's `side` face along axis a: the pair
    (v[m], v[m+1]) taken as the limit from the receiver's side.

    The potential on the receiver takes its data from the side its normal
    points to, i.e. the receiver's side (Lemma 2.2 and its one-sided
    convention; the 1 x 2 example of Sec. 3.2 uses n_i pointing into the
    receiving subdomain).  If this subdomain itself received a pair on the
    same face in the same sweep, its solution jumps there by that pair's
    field; the receiver-side continuation removes it: the layer on this
    subdomain's own side is reduced by the incoming pair's value on that
    layer, the other layer is kept."""
    dim = part.dim
    ax = dim - 1 - a
    m, m1 = _layers(part, a, side)
    vm = np.take(v, m, axis=ax).copy()
    vm1 = np.take(v, m1, axis=ax).copy()
    if incoming is not None:
        if side < 0:          # own side is layer m+1
            vm1 = vm1 - incoming[1]
        else:                 # own side is layer m
            vm = vm - incoming[0]
    return vm, vm1


def trace_source(part, S_r, pair, a, side):
    """g = [S_r, chi_r] v~ for a pair received on the receiver's `side` along
    axis a; chi_r is the receiver's half-space (its side of the interface)."""
    dim = part.dim
    ax = dim - 1 - a
    shp = part.ext_shape()
    m, m1 = _layers(part, a, side)
    vt = np.zeros(shp, dtype=complex)
    sl_m = [slice(None)] * dim
    sl_m[ax] = m
    sl_m1 = [slice(None)] * dim
    sl_m1[ax] = m1
    vt[tuple(sl_m)] = pair[0]
    vt[tuple(sl_m1)] = pair[1]
    chi = np.zeros(shp, dtype=float)
    sl = [slice(None)] * dim
    # receiver on the + side of the interface for its lower face, and on the
    # - side for its upper face
    sl[ax] = slice(m1, None) if side < 0 else slice(0, m + 1)
    chi[tuple(sl)] = 1.0
    vf = vt.ravel()
    cf = chi.ravel()
    g = S_r @ (cf * vf) - cf * (S_r @ vf)
    return g.reshape(shp)


def ddm_apply(prob, part, b, rounds=1, solvers=None, record=None,
              source_fn=None, route_fn=None):
    """u_DDM for the global right-hand side b (global-grid array, reversed-axis
    shape; in the layer it may be nonzero, as for a residual).

    rounds: number of rounds of the 2^n sweeps (2 = one extra round).
    record: optional list; (l, i, nonzero, ||u^l_i on owned nodes||) is
            appended for every (sweep, subdomain) slot.
    source_fn / route_fn: replacements of trace_source / route (tests plant
    mistakes through these to check that the DDM pins notice them)."""
    dim = prob.dim
    if solvers is None:
        solvers = SubdomainSolvers(part)
    source_fn = source_fn or trace_source
    route_fn = route_fn or route
    sweeps = sweep_directions(dim) * rounds
    u = np.zeros(prob.gshape, dtype=complex)
    # f_ij: the subdomain share of b on owned nodes, consumed at first use
    f_sub = {}
    for i in part.subdomains():
        g_sl, l_sl = part.owned_slices(i)
        fi = np.zeros(part.ext_shape(), dtype=complex)
        fi[l_sl] = b[g_sl]
        f_sub[i] = fi
    # traces[(l, i, a, side)] = [v_m, v_m1] accumulated pairs
    traces = {}
    for l, d in enumerate(sweeps):
        for group in step_groups(d, part.P):
            for i in group:
                S_r = solvers.ops[i]
                rhs = f_sub[i]
                f_sub[i] = np.zeros_like(rhs)          # set f_ij = 0
                rhs = rhs.copy()
                used = {}
                for a in range(dim):
                    for side in (-1, 1):
                        pair = traces.pop((l, i, a, side), None)
                        if pair is not None:
                            used[(a, side)] = pair
                            rhs += source_fn(part, S_r, pair, a, side)
                nonzero = bool(np.any(rhs != 0))
                if not nonzero:
                    if record is not None:
                        record.append((l, i, False, 0.0))
                    continue                           # u^l_ij = 0, no traces
                v = solvers.solve(i, rhs)
                g_sl, l_sl = part.owned_slices(i)
                u[g_sl] += v[l_sl]
                if record is not None:
                    record.append((l, i, True, float(np.linalg.norm(v[l_sl]))))
                for a in range(dim):
                    for side in (-1, 1):
                        j = list(i)
                        j[a] += side
                        if j[a] < 0 or j[a] >= part.P[a]:
                            continue
                        e = [0] * dim
                        e[a] = side
                        lp = route_fn(l, tuple(e), sweeps)
                        if lp is None:
                            continue
                        pair = extract_trace(part, v, a, side, used.get((a, side)))
                        key = (lp, tuple(j), a, -side)
                        if key in traces:
                            traces[key][0] = traces[key][0] + pair[0]
                            traces[key][1] = traces[key][1] + pair[1]
                        else:
                            traces[key] = [pair[0], pair[1]]
    return u
