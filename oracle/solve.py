"""Top-level oracle solvers.

solve_direct      u = A^{-1} f by SuperLU on the global padded-grid operator: the plain
                  definition of the discrete solution the method converges to.
solve_dd          Algorithm 5 in the full form: GMRES on A P y = f, u = P y (Sec. 2.3).
solve_dd_reduced  Algorithm 5 as printed: Algorithm 2, GMRES on the reduced columns with
                  Algorithm 3, then Algorithm 4.
solve_dd_concurrent  GMRES with the concurrent double sweep P_c (see dd.py), in the full form
                  or reduced to the columns where f - A P_c f lives.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import assemble_global
from .dd import (StripSolvers, apply_AP_concurrent_reduced, apply_AP_reduced, apply_P,
                 apply_P_concurrent, apply_P_reduced, concurrent_columns, reduced_setup,
                 reduced_setup_concurrent, to_reduced)
from .gmres import gmres_right
from .grid import Geometry


@dataclass
class Result:
    u: np.ndarray
    iters: int
    relres: float
    history: list


def relres(A, u: np.ndarray, f: np.ndarray) -> float:
    r = f.ravel() - A @ u.ravel()
    nf = np.linalg.norm(f.ravel())
    return float(np.linalg.norm(r) / nf) if nf > 0 else float(np.linalg.norm(r))


def solve_direct(g: Geometry, f: np.ndarray, A=None) -> np.ndarray:
    A = assemble_global(g) if A is None else A
    lu = spla.splu(A.tocsc(), permc_spec="COLAMD")
    if f.ndim == g.dim:
        return lu.solve(f.ravel().astype(np.complex128)).reshape(f.shape)
    return np.stack([lu.solve(fk.ravel().astype(np.complex128)).reshape(fk.shape) for fk in f])


def solve_dd(g: Geometry, f: np.ndarray, tol: float = 1e-6, maxit: int = 200,
             S: StripSolvers = None, A=None) -> Result:
    A = assemble_global(g) if A is None else A
    S = StripSolvers(g) if S is None else S
    op = lambda y: (A @ apply_P(g, S, A, y).ravel()).reshape(y.shape)
    y, it, hist = gmres_right(op, f, tol, maxit)
    u = apply_P(g, S, A, y)
    return Result(u, it, relres(A, u, f), hist)


def solve_dd_reduced(g: Geometry, f: np.ndarray, tol: float = 1e-6, maxit: int = 200,
                     S: StripSolvers = None, A=None) -> Result:
    A = assemble_global(g) if A is None else A
    S = StripSolvers(g) if S is None else S
    ut, phi = reduced_setup(g, S, A, f)                       # Algorithm 2
    if g.J == 1:
        return Result(ut, 0, relres(A, ut, f), [1.0])
    phi_r = to_reduced(g, phi)
    op = lambda psi: apply_AP_reduced(g, S, A, psi)           # Algorithm 3
    psi, it, hist = gmres_right(op, phi_r, tol, maxit)
    u = apply_P_reduced(g, S, A, psi, ut)                     # Algorithm 4
    return Result(u, it, relres(A, u, f), hist)


def solve_dd_concurrent(g: Geometry, f: np.ndarray, tol: float = 1e-6, maxit: int = 200,
                        S: StripSolvers = None, A=None, mode: str = "reduced") -> Result:
    A = assemble_global(g) if A is None else A
    S = StripSolvers(g) if S is None else S
    if mode == "full":
        op = lambda y: (A @ apply_P_concurrent(g, S, y).ravel()).reshape(y.shape)
        y, it, hist = gmres_right(op, f, tol, maxit)
        u = apply_P_concurrent(g, S, y)
        return Result(u, it, relres(A, u, f), hist)
    ut, phi = reduced_setup_concurrent(g, S, A, f)
    if g.J == 1:
        return Result(ut, 0, relres(A, ut, f), [1.0])
    cols = concurrent_columns(g)
    op = lambda psi: apply_AP_concurrent_reduced(g, S, A, psi)
    psi, it, hist = gmres_right(op, phi[..., cols].copy(), tol, maxit)
    full = np.zeros(g.field_shape, dtype=np.complex128)
    full[..., cols] = psi
    u = apply_P_concurrent(g, S, full) + ut
    return Result(u, it, relres(A, u, f), hist)


def solve_dd_robin(g: Geometry, f: np.ndarray, tol: float = 1e-6, maxit: int = 400,
                   R=None, A=None) -> Result:
    """GMRES with the Robin-transmission double sweep (Sec. 4.4), full form."""
    from .robin import RobinSolvers, apply_P_robin
    A = assemble_global(g) if A is None else A
    R = RobinSolvers(g) if R is None else R
    op = lambda y: (A @ apply_P_robin(g, R, A, y).ravel()).reshape(y.shape)
    y, it, hist = gmres_right(op, f, tol, maxit)
    u = apply_P_robin(g, R, A, y)
    return Result(u, it, relres(A, u, f), hist)


def solve_dd_concurrent_robin(g: Geometry, f: np.ndarray, tol: float = 1e-6, maxit: int = 400,
                              R=None, A=None) -> Result:
    """GMRES with the concurrent Robin sweeps of Sec. 3.1 (two-sided data, chains meeting in
    the middle), full form."""
    from .robin import RobinSolvers, apply_P_concurrent_robin
    A = assemble_global(g) if A is None else A
    R = RobinSolvers(g) if R is None else R
    op = lambda y: (A @ apply_P_concurrent_robin(g, R, A, y).ravel()).reshape(y.shape)
    y, it, hist = gmres_right(op, f, tol, maxit)
    u = apply_P_concurrent_robin(g, R, A, y)
    return Result(u, it, relres(A, u, f), hist)
