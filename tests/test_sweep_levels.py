"""CPU checks of the rule by which the library lets 2D sweep steps share a
launch, restated over the oracle's routing (Rules 2.4/2.5).

Subdomain s in sweep L reads its slot L, which each neighbour fills across
the shared face in every sweep L0 <= L that routes that face to L, and adds
into the slots of its neighbours.  The library puts (L, s) one level after
all of those writers and after (L - 1, s), and launches the steps whose
subdomains share a level together.  The checks: every slot's writers come
before its reader, the writers of one slot entry keep the sweep order of the
one-launch-per-step schedule (so every sum is added in the same order), a
step never spreads over two levels, and the launch counts are the ones the
GPU test expects of the library."""

import itertools

import pytest

import oracle.routing as R


def _subs(P):
    return [tuple(i) for i in itertools.product(range(P[0]), range(P[1]))]


def _writers(P, sweeps, L, s):
    """(L0, neighbour) pairs that add into slot L of s."""
    out = []
    for e in R.cardinal_directions(2):
        nb = (s[0] - e[0], s[1] - e[1])
        if not (0 <= nb[0] < P[0] and 0 <= nb[1] < P[1]):
            continue
        for L0 in range(L + 1):
            if R.route(L0, e, sweeps) == L:
                out.append((L0, nb))
    return out


def _levels(P, rounds):
    sweeps = R.sweep_directions(2) * rounds
    lev = {}
    for L, d in enumerate(sweeps):
        for group in R.step_groups(d, P):
            for s in group:
                v = lev[(L - 1, s)] + 1 if L > 0 else 0
                for w in _writers(P, sweeps, L, s):
                    v = max(v, lev[w] + 1)     # KeyError if a writer came later
                lev[(L, s)] = v
    return sweeps, lev


CASES = [((3, 3), 2, 40, 32), ((1, 4), 2, 32, 20), ((3, 5), 2, 56, 40),
         ((4, 1), 1, 16, 16), ((2, 2), 1, 12, 10), ((8, 8), 1, 60, 46),
         ((16, 16), 2, 248, 188), ((32, 32), 2, 504, 380)]


@pytest.mark.parametrize("P,rounds,per_step,merged", CASES)
def test_levels_order_every_slot(P, rounds, per_step, merged):
    sweeps, lev = _levels(P, rounds)
    for (L, s), v in lev.items():
        # the slot is complete before it is read
        assert all(lev[w] < v for w in _writers(P, sweeps, L, s))
    # the writers of one slot entry (slot lq of r across direction e) add
    # in sweep order
    for lq in range(len(sweeps)):
        for r in _subs(P):
            for e in R.cardinal_directions(2):
                nb = (r[0] - e[0], r[1] - e[1])
                if not (0 <= nb[0] < P[0] and 0 <= nb[1] < P[1]):
                    continue
                ws = [L0 for L0 in range(len(sweeps)) if R.route(L0, e, sweeps) == lq]
                vs = [lev[(L0, nb)] for L0 in ws]
                assert vs == sorted(vs) and len(set(vs)) == len(vs)


@pytest.mark.parametrize("P,rounds,per_step,merged", CASES)
def test_whole_steps_share_levels(P, rounds, per_step, merged):
    sweeps, lev = _levels(P, rounds)
    step_level = {}
    for L, d in enumerate(sweeps):
        for st, group in enumerate(R.step_groups(d, P)):
            vs = {lev[(L, s)] for s in group}
            assert len(vs) == 1                   # a step stays whole
            step_level[(L, st)] = vs.pop()
    assert len(step_level) == per_step
    by_level = {}
    for k, v in step_level.items():
        by_level.setdefault(v, []).append(k)
    assert len(by_level) == merged
    # at most two steps, of different sweeps, per launch
    for steps in by_level.values():
        assert len(steps) <= 2 and len({L for L, _ in steps}) == len(steps)


def test_planted_missing_writer_is_caught():
    # without the previous-sweep link the writers of one entry can share a
    # level, which the order check refuses
    P, rounds = (3, 3), 2
    sweeps = R.sweep_directions(2) * rounds
    lev = {}
    for L, d in enumerate(sweeps):
        for group in R.step_groups(d, P):
            for s in group:
                v = 0
                for w in _writers(P, sweeps, L, s):
                    v = max(v, lev[w] + 1)
                lev[(L, s)] = v
    clash = False
    for lq in range(len(sweeps)):
        for r in _subs(P):
            for e in R.cardinal_directions(2):
                nb = (r[0] - e[0], r[1] - e[1])
                if not (0 <= nb[0] < P[0] and 0 <= nb[1] < P[1]):
                    continue
                vs = [lev[(L0, nb)] for L0 in range(len(sweeps))
                      if R.route(L0, e, sweeps) == lq]
                clash |= vs != sorted(vs) or len(set(vs)) != len(vs)
    assert clash
