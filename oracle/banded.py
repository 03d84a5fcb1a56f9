"""Direct solvers of the oracle.

The paper factors every subdomain problem once with a sparse direct solver and
reuses the factors for every solve (Sec. 5); the oracle does the same with
LAPACK's banded LU with partial pivoting (zgbtrf / zgbtrs).  With x-fastest
ordering the bandwidth of the 5-point (7-point) operator is the node count of
one x-line (one xy-plane).
"""

import numpy as np
import scipy.sparse.linalg as spla
from scipy.linalg.lapack import zgbtrf, zgbtrs

from .discretization import global_operator


class BandedLU:
    """Banded LU factor of a complex sparse matrix with half-bandwidth kb."""

    def __init__(self, S, kb):
        S = S.tocoo()
        n = S.shape[0]
        kl = ku = int(kb)
        assert np.all(np.abs(S.row - S.col) <= kb), "matrix exceeds band"
        ab = np.zeros((2 * kl + ku + 1, n), dtype=complex)
        ab[kl + ku + S.row - S.col, S.col] = S.data
        lu, piv, info = zgbtrf(ab, kl, ku)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrf info={info}")
        self.lu, self.piv, self.kl, self.ku, self.n = lu, piv, kl, ku, n

    def solve(self, B):
        B = np.asarray(B, dtype=complex)
        vec = B.ndim == 1
        B2 = B.reshape(self.n, -1)
        X, info = zgbtrs(self.lu, self.kl, self.ku, B2, self.piv)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrs info={info}")
        return X.reshape(B.shape) if not vec else X[:, 0]


def band_of(shape):
    """Half-bandwidth of the stencil operator on a reversed-axis grid shape:
    the stride of the slowest axis."""
    return int(np.prod(shape[1:]))


def solve_global(prob, b, method="auto"):
    """u_glob = S^{-1} b for the global PML problem (the plain definition of
    the solution the DDM is proved to reproduce, Thm 3.3 / Thm 3.10).

    b: global-grid array (reversed-axis shape) or a stack of them along a
    leading axis.  method 'banded' (LAPACK band LU), 'sparse' (SuperLU), or
    'auto' (banded when the band storage stays below ~2 GB)."""
    S = global_operator(prob)
    gshape = prob.gshape
    b = np.asarray(b, dtype=complex)
    stacked = b.ndim == len(gshape) + 1
    B = b.reshape(-1, int(np.prod(gshape))).T
    kb = band_of(gshape)
    if method == "auto":
        method = "banded" if (3 * kb + 1) * S.shape[0] * 16 < 2e9 else "sparse"
    if method == "banded":
        X = BandedLU(S, kb).solve(B)
    else:
        lu = spla.splu(S.tocsc())
        X = lu.solve(B)
    X = X.T.reshape((-1,) + gshape)
    return X if stacked else X[0]
