"""FP64 Krylov drivers around the DDM (Sec. 5.2: the DDM used as a
preconditioner for GMRES, stopping on the relative residual).

* refine: x_{j+1} = x_j + M^{-1}(b - S x_j), stopping when
  ||b - S x|| / ||b|| <= tol.
* gmres: right-preconditioned restarted GMRES(m), modified Gram-Schmidt
  Arnoldi, Givens rotations on the Hessenberg matrix, the same stopping test
  on the true residual at every restart.

S is a scipy sparse matrix (or anything with @), M a callable on flat
vectors.  Both return (x, history of relative residuals); gmres's history
holds the true residual at every restart, and its optional `info` dict
receives the total number of Arnoldi steps ("iters") and the residual
estimate after every step ("estimates").
"""

import numpy as np


def refine(S, b, M, tol=1e-10, maxit=50):
    b = np.asarray(b, dtype=complex).ravel()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = []
    for _ in range(maxit + 1):
        r = b - S @ x
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= tol:
            break
        x = x + M(r)
    return x, hist


def gmres(S, b, M, m=20, tol=1e-10, maxit=200, info=None):
    b = np.asarray(b, dtype=complex).ravel()
    nb = np.linalg.norm(b)
    n = b.size
    x = np.zeros_like(b)
    hist = []
    est = []
    it = 0
    while True:
        r = b - S @ x
        beta = np.linalg.norm(r)
        hist.append(beta / nb)
        if beta / nb <= tol or it >= maxit:
            break
        V = np.zeros((m + 1, n), dtype=complex)
        Z = np.zeros((m, n), dtype=complex)
        H = np.zeros((m + 1, m), dtype=complex)
        cs = np.zeros(m, dtype=complex)
        sn = np.zeros(m, dtype=complex)
        g = np.zeros(m + 1, dtype=complex)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(m):
            Z[k] = M(V[k])
            w = S @ Z[k]
            for j in range(k + 1):                 # modified Gram-Schmidt
                H[j, k] = np.vdot(V[j], w)
                w = w - H[j, k] * V[j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0:
                V[k + 1] = w / H[k + 1, k]
            for j in range(k):                     # apply previous rotations
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -np.conj(sn[j]) * H[j, k] + np.conj(cs[j]) * H[j + 1, k]
                H[j, k] = t
            a, bb = H[k, k], H[k + 1, k]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0:
                cs[k], sn[k] = 1.0, 0.0
            else:
                cs[k] = a / den
                sn[k] = bb / den
                cs[k], sn[k] = np.conj(cs[k]), np.conj(sn[k])
            H[k, k] = cs[k] * a + sn[k] * bb
            H[k + 1, k] = 0.0
            g[k + 1] = -np.conj(sn[k]) * g[k]
            g[k] = cs[k] * g[k]
            k_used = k + 1
            it += 1
            est.append(abs(g[k + 1]) / nb)
            if abs(g[k + 1]) / nb <= tol or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + y @ Z[:k_used]
    if info is not None:
        info["iters"] = it
        info["estimates"] = est
    return x, hist
