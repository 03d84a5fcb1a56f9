"""Pins of the sweep schedule and trace routing against the hand-derived
tables of Rules 2.4/2.5 and 4.1/4.2 and the step structure of eq. (step_subd)
and eq. (step_subd3)."""

import os

import numpy as np
import pytest

import oracle as O
from oracle.routing import cardinal_directions

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(v) for v in line.split()])
    return rows


def test_routing_table_2d_matches_hand_derivation():
    assert O.routing_table(2, rounds=2) == _load("routing_2d.txt")


def test_routing_table_3d_matches_hand_derivation():
    assert O.routing_table(3, rounds=2) == _load("routing_3d.txt")


def test_single_round_drops_late_traces():
    # With one round, traces whose admissible sweep lies in a next round
    # are dropped.
    sweeps = O.sweep_directions(2)
    assert O.route(1, (1, 0), sweeps) is None
    assert O.route(3, (0, 1), sweeps) is None
    assert O.route(0, (-1, 0), sweeps) == 1


@pytest.mark.parametrize("P", [(5, 5), (3, 7), (1, 4), (2, 3, 4), (3, 3, 3)])
def test_step_groups(P):
    dim = len(P)
    for d in O.sweep_directions(dim):
        groups = O.step_groups(d, P)
        assert len(groups) == sum(P) - dim + 1
        seen = sorted(i for g in groups for i in g)
        assert len(seen) == int(np.prod(P)) and len(set(seen)) == len(seen)
        # the sweep starts at the corner opposite to d and every subdomain's
        # upwind neighbours (along d) are in the previous step
        for s, g in enumerate(groups):
            for i in g:
                for a in range(dim):
                    j = list(i)
                    j[a] -= d[a]
                    if 0 <= j[a] < P[a]:
                        assert tuple(j) in groups[s - 1]


def test_rules_used_traces_once_per_round():
    # every direction of every sweep is routed to a sweep whose direction is
    # similar to it (Rule 2.4 / 4.1) or dropped
    for dim in (2, 3):
        sweeps = O.sweep_directions(dim) * 2
        for l in range(len(sweeps)):
            for e in cardinal_directions(dim):
                lp = O.route(l, e, sweeps)
                if lp is not None:
                    assert O.similar(e, sweeps[lp])
                    assert lp >= l
