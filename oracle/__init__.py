"""Plain FP64 CPU oracle for the trace-transfer diagonal sweeping DDM
(Leng & Ju, "Trace transfer-based diagonal sweeping DDM for the Helmholtz
equation: algorithms and convergence analysis", arXiv:2003.02585).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under this package: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use
it.  It shares no code with the HIP path.

What it computes (all complex128 / float64):

* ``discretization``  -- grid, uniaxial PML stretching (Sec. 2.1, eq. sigma
  and the coordinate stretching after it), the J-scaled 5-/7-point operator
  discretizing eq. (PML) / eq. (PML3), and the right-hand side b = h^2 J f.
* ``banded``          -- LAPACK banded LU (zgbtrf / zgbtrs), the direct
  solver for the global problem and for every subdomain problem.
* ``routing``         -- sweep orders (Sorder2D, Sorder3D), step groups
  (eq. step_subd, step_subd3) and the trace routing of Rules 2.4/2.5
  (2D) and 4.1/4.2 (3D).
* ``ddm``             -- Algorithm 2.1 (2D) and Algorithm 4.1 (3D), step by
  step, with the discrete trace potential realised as the commutator
  source [S_r, chi_r] v (Lemma 2.2 in discrete form).
* ``krylov``          -- FP64 iterative refinement and right-preconditioned
  GMRES(m) with the DDM as preconditioner (Sec. 5.2).

Every function's docstring names the passage of the paper it follows.
"""

from .discretization import (Problem, Partition, sigma0_from_R, alpha,
                             assemble, global_operator, global_rhs)
from .banded import BandedLU, solve_global
from .routing import (sweep_directions, step_groups, route, routing_table,
                      similar, opposite_blocked)
from .ddm import ddm_apply, SubdomainSolvers
from .krylov import refine, gmres

__all__ = [
    "Problem", "Partition", "sigma0_from_R", "alpha", "assemble",
    "global_operator", "global_rhs", "BandedLU", "solve_global",
    "sweep_directions", "step_groups", "route", "routing_table", "similar",
    "opposite_blocked", "ddm_apply", "SubdomainSolvers", "refine", "gmres",
]
