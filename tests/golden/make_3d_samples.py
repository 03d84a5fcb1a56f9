"""Write sampled oracle values for the 3D parity tests at the real plane-block
size of the 96^3 workload (n_ext = 44, a block of 44^2 = 1936 nodes per
plane, K = 44 planes per subdomain).  Calls only the oracle and the seeded
input module.

python tests/golden/make_3d_samples.py ddm_c4block
    One DDM application (Algorithm 4.1, one round of 8 sweeps, FP64 banded
    subdomain solves) on a 64^3 grid, W = 6, 2 x 2 x 2 subdomains of 32^3
    (so every subdomain is extended to 44^3, the block size of the 96^3
    workload), constant k at 8 points per wavelength, for the b-space
    vectors b = h^2 J f of two seeded Gaussian sources.  Stores u_DDM at 4096
    seeded global nodes and its 2-norm over the global grid, per RHS.
    -> tests/golden/ddm_c4block.npz

python tests/golden/make_3d_samples.py glob_c3d
    The global PML solution of the 96^3 workload (3 x 3 x 3, W = 6, 8 ppw)
    for its first two sources, computed as the oracle's right-preconditioned
    FP64 GMRES(20) with the oracle's DDM as preconditioner, to a relative
    residual of 1e-13 (the global band LU would need ~700 GB).  Stores u at
    256 seeded interior nodes, the interior 2-norm, the final residual and
    the residual history.
    -> tests/golden/glob_c3d.npz
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                   # noqa: E402
from paper_2003_02585_amd import workloads as wl     # noqa: E402


def c4block_workload():
    """The 2 x 2 x 2 case with 32^3 subdomains: the c3d recipe at N = 64."""
    return wl.make("c3d", N=64, P=2, nrhs=2)


def ddm_c4block():
    w = c4block_workload()
    prob = O.Problem(w["kappa"], w["h"], w["W"])
    part = O.Partition(prob, w["P"])
    t0 = time.time()
    solvers = O.SubdomainSolvers(part)
    print(f"ddm_c4block: {solvers.n_distinct} distinct operator(s) factored in "
          f"{time.time() - t0:.1f} s", flush=True)
    gsize = int(np.prod(prob.gshape))
    rng = np.random.default_rng(20030258)
    idx = np.sort(rng.choice(gsize, size=4096, replace=False))
    vals, norms = [], []
    for j, fj in enumerate(w["f"]):
        t0 = time.time()
        b = O.global_rhs(prob, fj)
        u = O.ddm_apply(prob, part, b, solvers=solvers).ravel()
        vals.append(u[idx])
        norms.append(np.linalg.norm(u))
        print(f"ddm_c4block: RHS {j} applied in {time.time() - t0:.1f} s", flush=True)
    out = os.path.join(HERE, "ddm_c4block.npz")
    np.savez_compressed(out, index=idx, values=np.array(vals), norms=np.array(norms),
                        pml_R=np.float64(1e-16))
    print(f"ddm_c4block: wrote {out}", flush=True)


class NearDedupSolvers(O.SubdomainSolvers):
    """Subdomain operators that agree to rounding share one banded factor.

    The oracle computes each subdomain's layer profile from absolute
    coordinates, so translated copies of one operator can differ in the last
    bits (at 96^3 the 27 copies would need 27 factors of 7.9 GB).  Here the
    DDM is only GMRES's preconditioner: the GMRES answer S^-1 b, with S the
    exact global operator, does not depend on it."""

    def __init__(self, part, rtol=1e-13):
        self.part = part
        self.ops, self.key, self.factors = {}, {}, {}
        kb = O.banded.band_of(part.ext_shape())
        reps = []
        for i in part.subdomains():
            S = part.operator(i).tocsr()
            S.sort_indices()
            self.ops[i] = S
            key = None
            for k, R in reps:
                if (np.array_equal(S.indptr, R.indptr) and np.array_equal(S.indices, R.indices)
                        and np.max(np.abs(S.data - R.data)) <= rtol * np.max(np.abs(R.data))):
                    key = k
                    break
            if key is None:
                key = len(reps)
                reps.append((key, S))
                self.factors[key] = O.BandedLU(S, kb)
            self.key[i] = key


def glob_c3d(nrhs=2, tol=1e-13):
    w = wl.make("c3d")
    prob = O.Problem(w["kappa"], w["h"], w["W"])
    part = O.Partition(prob, w["P"])
    S = O.global_operator(prob).tocsr()
    t0 = time.time()
    solvers = NearDedupSolvers(part)
    print(f"glob_c3d: {solvers.n_distinct} distinct operator(s) factored in "
          f"{time.time() - t0:.1f} s", flush=True)
    gshape = prob.gshape
    count = [0]

    def M(r):
        count[0] += 1
        t1 = time.time()
        z = O.ddm_apply(prob, part, r.reshape(gshape), solvers=solvers).ravel()
        print(f"glob_c3d:   DDM application {count[0]} in {time.time() - t1:.1f} s",
              flush=True)
        return z

    N = w["kappa"].shape
    rng = np.random.default_rng(20030258)
    flat = rng.choice(int(np.prod(N)), size=256, replace=False)
    sl = prob.interior_slice()
    vals = np.zeros((nrhs, 256), dtype=complex)
    norms = np.zeros(nrhs)
    resid = np.zeros(nrhs)
    hists = []
    for j in range(nrhs):
        b = O.global_rhs(prob, w["f"][j]).ravel()
        u, hist = O.gmres(S, b, M, m=20, tol=tol, maxit=60)
        resid[j] = np.linalg.norm(b - S @ u) / np.linalg.norm(b)
        ui = u.reshape(gshape)[sl].ravel()
        vals[j] = ui[flat]
        norms[j] = np.linalg.norm(ui)
        hists.append(np.array(hist))
        print(f"glob_c3d: RHS {j}: residual {resid[j]:.2e} after {len(hist) - 1} restarts, "
              f"history {[f'{h:.1e}' for h in hist]}", flush=True)
    out = os.path.join(HERE, "glob_c3d.npz")
    np.savez_compressed(out, index=flat, values=vals, norms=norms, residual=resid,
                        pml_R=np.float64(1e-16))
    print(f"glob_c3d: wrote {out}; max residual {resid.max():.2e}", flush=True)


if __name__ == "__main__":
    {"ddm_c4block": ddm_c4block, "glob_c3d": glob_c3d}[sys.argv[1]]()
