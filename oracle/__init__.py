"""CPU FP64 oracle for the PML-transmission double-sweep Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import or run anything in this package.
The product path (`paper_1208_3956_amd`) never imports it, and this package never
imports the product path: the two share no code.  Inputs come from the
`workloads` module, which holds none of the method's arithmetic.

Everything here is plain, slow and written to be checked against the paper by eye:
scipy sparse matrices in complex128, SuperLU (`splu`) for every solve, and the
sweeps and GMRES written step by step in the paper's order.

Modules
  grid      padded grid, partition of the x axis, PML coefficient tables
  assemble  the finite-difference operator A and the padded strip operators A^(j)
  dd        double-sweep preconditioner P (full form) and the reduced form
  gmres     right-preconditioned GMRES
  greens    discrete free-space Green's function of the 5-point lattice
  grad      misfit and its gradient with respect to squared slowness
"""
from .grid import Geometry, make_geometry
from .assemble import assemble_global, assemble_strip, apply_A
from .dd import StripSolvers, apply_P, apply_AP_full, reduced_setup, apply_AP_reduced, apply_P_reduced
from .gmres import gmres_right
from .solve import solve_direct, solve_dd, solve_dd_reduced

__all__ = [
    "Geometry", "make_geometry", "assemble_global", "assemble_strip", "apply_A",
    "StripSolvers", "apply_P", "apply_AP_full", "reduced_setup", "apply_AP_reduced",
    "apply_P_reduced", "gmres_right", "solve_direct", "solve_dd", "solve_dd_reduced",
]
