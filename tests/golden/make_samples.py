"""Write sampled values of the global PML solution u_glob = S^{-1} b for the
full-size workloads (FP64 oracle: SuperLU with two steps of FP64 iterative
refinement), for full-size GPU parity tests.

Calls only the oracle and the seeded input module.  For every RHS of the
workload it stores u_glob at 256 interior nodes drawn with a fixed seed and
the 2-norm of u_glob over the interior nodes.

python tests/golden/make_samples.py c2d      -> tests/golden/samples_c2d.npz
python tests/golden/make_samples.py layer2d  -> tests/golden/samples_layer2d.npz
"""
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                   # noqa: E402
from paper_2003_02585_amd import workloads as wl     # noqa: E402

NSAMP = 256


def main(name):
    w = wl.make(name)
    prob = O.Problem(w["kappa"], w["h"], w["W"])
    t0 = time.time()
    S = O.global_operator(prob).tocsc()
    lu = spla.splu(S, permc_spec="COLAMD")
    print(f"{name}: factor {time.time() - t0:.1f} s", flush=True)
    N = w["kappa"].shape
    rng = np.random.default_rng(20030258)
    flat = rng.choice(int(np.prod(N)), size=NSAMP, replace=False)
    sl = prob.interior_slice()
    vals = np.zeros((len(w["f"]), NSAMP), dtype=complex)
    norms = np.zeros(len(w["f"]))
    resid = np.zeros(len(w["f"]))
    for j, fj in enumerate(w["f"]):
        b = O.global_rhs(prob, fj).ravel()
        u = lu.solve(b)
        for _ in range(2):
            # FP64 iterative refinement of the direct solve
            u = u + lu.solve(b - S @ u)
        resid[j] = np.linalg.norm(b - S @ u) / np.linalg.norm(b)
        ui = u.reshape(prob.gshape)[sl].ravel()
        vals[j] = ui[flat]
        norms[j] = np.linalg.norm(ui)
    out = os.path.join(HERE, f"samples_{name}.npz")
    np.savez_compressed(out, index=flat, values=vals, norms=norms, residual=resid,
                        pml_R=np.float64(1e-16))
    print(f"{name}: wrote {out}; max oracle residual {resid.max():.2e}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
