"""Sweep order, step groups and trace routing.

* Sweep order: eq. (Sorder2D) in 2D, eq. (Sorder3D) in 3D.
* Step groups: eq. (step_subd)/(step_subd_ij) in 2D and eq. (step_subd3)/
  (step_subd_k) in 3D -- step s of the sweep in direction d holds the
  subdomains with sum_a ihat_a(i_a) + 1 = s, ihat_a = i_a (d_a = +1) or
  P_a - 1 - i_a (d_a = -1) with 0-based i.
* Routing (Algorithm 2.1 / 4.1): a trace generated in sweep l travelling in
  direction e is added to the trace slot of the smallest sweep l' >= l in
  which it may be used by
    - Rule 2.4 / 4.1 (similar directions): only in a sweep d with e.d > 0
      (3D additionally e_k d_k >= 0 for every k);
    - Rule 2.5 (2D, opposite directions): never in a later sweep whose
      direction is the opposite of the generating sweep's;
    - Rule 4.2 (3D): never in a later sweep d2 if, in one of the xy, xz, yz
      coordinate-plane projections, the projection of e has exactly one zero
      component and the projections of the generating sweep d1 and of d2 are
      opposite.  (The paper words Rule 4.2 for transferred sources; the
      oracle applies it to traces.)
  With more than one round the sweep list is the order repeated, and the
  rules are applied over the whole extended list, so traces the first round
  cannot use are carried into the next round (the extra round of Thm 3.6,
  Thm 3.10 and Sec. 4).  A trace with no admissible sweep is dropped.
"""

import itertools

import numpy as np


def sweep_directions(dim):
    """Sorder2D / Sorder3D, as tuples (d_x, d_y[, d_z])."""
    if dim == 2:
        return [(1, 1), (-1, 1), (1, -1), (-1, -1)]
    if dim == 3:
        out = []
        for dz in (1, -1):
            for dy in (1, -1):
                for dx in (1, -1):
                    out.append((dx, dy, dz))
        return out
    raise ValueError("dim must be 2 or 3")


def similar(e, d):
    """Similar directions: e.d > 0, and in 3D also e_k d_k >= 0 for all k."""
    dot = sum(a * b for a, b in zip(e, d))
    if dot <= 0:
        return False
    if len(e) == 3:
        return all(a * b >= 0 for a, b in zip(e, d))
    return True


def opposite_blocked(e, d_gen, d_use):
    """True if Rule 2.5 (2D) / Rule 4.2 (3D) forbids using a trace of direction
    e generated in a sweep of direction d_gen in a LATER sweep d_use."""
    dim = len(e)
    if dim == 2:
        return tuple(d_use) == tuple(-v for v in d_gen)
    for (a, b) in ((0, 1), (0, 2), (1, 2)):
        pe = (e[a], e[b])
        if sum(1 for v in pe if v == 0) != 1:
            continue
        if (d_use[a], d_use[b]) == (-d_gen[a], -d_gen[b]):
            return True
    return False


def route(l, e, sweeps):
    """Smallest l' >= l (0-based, over the extended list `sweeps`) in which a
    trace of direction e generated in sweep l may be used; None if none."""
    for lp in range(l, len(sweeps)):
        if not similar(e, sweeps[lp]):
            continue
        if lp > l and opposite_blocked(e, sweeps[l], sweeps[lp]):
            continue
        return lp
    return None


def cardinal_directions(dim):
    """Trace directions in the order +x, -x, +y, -y(, +z, -z)."""
    out = []
    for a in range(dim):
        for s in (1, -1):
            e = [0] * dim
            e[a] = s
            out.append(tuple(e))
    return out


def routing_table(dim, rounds=2):
    """Table[l][k] = l' (1-based, as printed in the paper's numbering) for
    sweep l of the first round and the k-th cardinal direction; 0 = dropped."""
    sweeps = sweep_directions(dim) * rounds
    tab = []
    for l in range(len(sweep_directions(dim))):
        row = []
        for e in cardinal_directions(dim):
            lp = route(l, e, sweeps)
            row.append(0 if lp is None else lp + 1)
        tab.append(row)
    return tab


def step_index(i, d, P):
    """s for subdomain i (0-based) in the sweep of direction d (1-based s)."""
    s = 1
    for a in range(len(P)):
        s += i[a] if d[a] == 1 else P[a] - 1 - i[a]
    return s


def step_groups(d, P):
    """List over steps s = 1 .. sum(P) - dim + 1 of the subdomains solved at
    step s of the sweep in direction d."""
    dim = len(P)
    nsteps = sum(P) - dim + 1
    groups = [[] for _ in range(nsteps)]
    for i in itertools.product(*[range(p) for p in P]):
        groups[step_index(i, d, P) - 1].append(tuple(i))
    return groups
