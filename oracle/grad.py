"""Misfit and its gradient with respect to squared slowness (oracle).

Not part of the paper: the differentiation form of the solver.  With m = 1/c^2 on the
interior, k^2 = omega^2 m (continued into the outer PML by the nearest interior value),
sources f_s, receivers R (a list of padded-grid points) and data d_s,
    J(m) = 1/2 sum_s || R u_s - d_s ||^2,   A(m) u_s = f_s.
Since only the -k^2 u term of A depends on m, dA/dm_p = -omega^2 sum_{q -> p} e_q e_q^T
(q runs over the padded points whose medium is taken from interior point p), and
    dJ/dm_p = omega^2 Re sum_s sum_{q -> p} conj(lambda_s[q]) u_s[q],
    A^H lambda_s = R^T (R u_s - d_s).
The oracle solves the adjoint systems with a direct factorisation of A^H (no use of
the complex symmetry of D^{-1} A).  The PML is held fixed: c_ref is given explicitly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import assemble_global
from .grid import make_geometry


def _geometry(g0, m):
    c = 1.0 / np.sqrt(m)
    return make_geometry(c, g0.omega, g0.h, g0.w_out, g0.w, g0.J, g0.power, g0.s0,
                         beta=list(g0.beta[1:-1]), cref=g0.c_ref)


def misfit(g0, m, f, rec, d):
    """J(m) and the fields u_s (direct solves).  f: (nsrc, N_y, N_x); rec: flat padded
    indices; d: (nsrc, nrec)."""
    g = _geometry(g0, m)
    A = assemble_global(g).tocsc()
    lu = spla.splu(A, permc_spec="COLAMD")
    U = np.stack([lu.solve(fs.ravel().astype(np.complex128)) for fs in f])
    r = U[:, rec] - d
    return 0.5 * float(np.sum(np.abs(r) ** 2)), U


def gradient(g0, m, f, rec, d):
    """(J, dJ/dm) by the adjoint-state method with direct solves."""
    g = _geometry(g0, m)
    A = assemble_global(g).tocsc()
    lu = spla.splu(A, permc_spec="COLAMD")
    luH = spla.splu(A.conj().T.tocsc(), permc_spec="COLAMD")
    grad = np.zeros(m.size)
    clamp = g.clamp_index().ravel()
    Jval = 0.0
    for fs, ds in zip(f, d):
        u = lu.solve(fs.ravel().astype(np.complex128))
        r = u[rec] - ds
        Jval += 0.5 * float(np.sum(np.abs(r) ** 2))
        q = np.zeros_like(u)
        np.add.at(q, rec, r)
        lam = luH.solve(q)
        contrib = g.omega ** 2 * np.real(np.conj(lam) * u)
        np.add.at(grad, clamp, contrib)
    return Jval, grad.reshape(m.shape)
