"""CPU model of the 3D factorization's two-level blocked Gauss-Jordan
inversion (the steps the HIP kernels take, in NumPy): register panels whose
pivots become row interchanges only at the panel's end, a list of row
moves per panel applied to the other columns, inner updates confined to the
outer panel, one rank-OB update of the rest, and the column order restored
from the interchanges.  The model must reproduce the inverse to rounding
for panel widths that do and do not divide the block size, and its
pivoting must survive a zero leading entry."""

import numpy as np
import pytest


def _key(m, row):
    # |Re| + |Im| with its exponent and leading 10 mantissa bits, then the
    # lowest row (the kernels' 32-bit key)
    b = int(np.float32(m).view(np.uint32))
    return (b & ~8191) | (8191 - row)


def _panel(A, j0, nbr, piv):
    n = A.shape[0]
    P = A[:, j0:j0 + nbr].copy()
    cand = np.arange(n) >= j0
    chosen = []
    for q in range(nbr):
        keys = [_key(abs(P[i, q].real) + abs(P[i, q].imag), i) if cand[i] else 0
                for i in range(n)]
        p = 8191 - (max(keys) & 8191)
        inv = 1 / P[p, q]
        scaled = np.array([inv if c == q else P[p, c] * inv for c in range(nbr)])
        for i in range(n):
            if i != p:
                f = P[i, q]
                P[i] = P[i] - f * scaled
                P[i, q] = -f * inv
        P[p] = scaled
        cand[p] = False
        chosen.append(p)
    # interchanges of the swapping algorithm and the net moves of the rows
    moved = {}                                # row -> final position
    for q, p in enumerate(chosen):
        a = j0 + q
        rq = moved.get(p, p)
        y = next((r for r, pos in moved.items() if pos == a), a)
        piv[a] = rq
        if rq != a:
            moved[p] = a
            moved[y] = rq
    for i in range(n):
        A[moved.get(i, i), j0:j0 + nbr] = P[i]
    return [(pos, row) for row, pos in moved.items()]   # (destination, source)


def _apply_moves(col, moves):
    vals = [col[s] for _, s in moves]
    for (d, _), v in zip(moves, vals):
        col[d] = v


def gj_two_level(D, nb, ob):
    n = D.shape[0]
    A = D.astype(complex).copy()
    piv = np.zeros(n, int)
    for J0 in range(0, n, ob):
        OBr = min(ob, n - J0)
        lists = []
        for j0 in range(J0, J0 + OBr, nb):
            nbr = min(nb, J0 + OBr - j0)
            mv = _panel(A, j0, nbr, piv)
            lists.append(mv)
            E = A[:, j0:j0 + nbr].copy()
            for j in range(J0, J0 + OBr):
                if j0 <= j < j0 + nbr:
                    continue
                col = A[:, j]
                _apply_moves(col, mv)
                r = col[j0:j0 + nbr].copy()
                col[j0:j0 + nbr] = 0
                col += E @ r
        R = np.zeros((OBr, n), complex)
        for j in range(n):
            if J0 <= j < J0 + OBr:
                continue
            col = A[:, j]
            for mv in lists:
                _apply_moves(col, mv)
            R[:, j] = col[J0:J0 + OBr]
            col[J0:J0 + OBr] = 0
        E = A[:, J0:J0 + OBr].copy()
        mask = np.ones(n, bool)
        mask[J0:J0 + OBr] = False
        A[:, mask] += E @ R[:, mask]
    for kc in range(n - 1, -1, -1):
        r = piv[kc]
        A[:, [kc, r]] = A[:, [r, kc]]
    return A


@pytest.mark.parametrize("n,nb,ob", [(37, 16, 128), (70, 16, 32), (50, 8, 16), (130, 16, 64),
                                     (20, 8, 128)])
def test_two_level_model_inverts(n, nb, ob):
    rng = np.random.default_rng(n)
    D = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    X = gj_two_level(D, nb, ob)
    assert np.abs(X @ D - np.eye(n)).max() < 1e-10


def test_two_level_model_pivots_past_a_zero_diagonal():
    # a zero leading entry (and zero diagonal) forces interchanges in every
    # panel: a complex symmetric block of the kind the factorization sees
    rng = np.random.default_rng(3)
    n = 48
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    D = B + B.T
    np.fill_diagonal(D, 0)
    X = gj_two_level(D, 16, 32)
    assert np.abs(X @ D - np.eye(n)).max() < 1e-9
