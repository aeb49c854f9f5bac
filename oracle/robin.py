"""The double sweep with Robin transmission conditions (oracle), the paper's comparison
method (Sec. 4.4, Tables 4 and 5).

Subdomain j covers the columns of D^(j) plus the shifted boundary's extra column (the
overlap of one grid point, m_overlap = 1), with no PML pads: its internal sides carry
Robin conditions instead.  The right (upward) sweep solves, for j = 1..J,
    -Laplace v^(j) - k^2 v^(j) = f^(j)                      on the subdomain,
     d_x v^(j) + i k v^(j) =  d_x v^(j-1) + i k v^(j-1)     at its left side,
    -d_x v^(j) + i k v^(j) = 0                              at its right side,
with f^(j) = f on D^(j), and v = v^(j) on D^(j); the left (downward) sweep is its mirror
image on the residual g = f - A v (right side fed by w^(j+1), left side homogeneous,
g^(j) = g on D~^(j), w = w^(j) on D~^(j)); the preconditioner is v + w.  The outer PML and
the y-PML are those of the global operator.

Discretisation (the paper gives none; a reading): a Robin condition sits at the half-point
between the boundary column b and a ghost column outside; d_x is the two-point difference
and u the two-point mean there, so the ghost value is rho u_b - (data) / (1/h - i k/2) with
rho = (1 + i k h/2) / (1 - i k h/2), k taken at the boundary column.  Eliminating the ghost
adds -alpha_x(b) alpha_x(b +- 1/2) rho / h^2 to the diagonal of column b and moves the data
to the right-hand side; with the data of a neighbour field V at the two columns next to the
half-point (inner column V_i, outer column V_o) the right-hand side of column b gains
(V_o - rho V_i) / h^2 (alpha = 1 at internal boundaries).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import assemble_5pt
from .grid import Geometry


def robin_rho(g: Geometry, col: int) -> np.ndarray:
    """rho = (1 + i k h/2) / (1 - i k h/2) on every row, k at global column col."""
    k = np.sqrt(g.k2()[..., col])
    return (1 + 0.5j * k * g.h) / (1 - 0.5j * k * g.h)


def robin_span(g: Geometry, s: int):
    """[lo, hi) global columns of Robin subdomain s: the core and the extra column."""
    st = g.strips[s]
    return st.dom


def assemble_robin_strip(g: Geometry, s: int) -> sp.csr_matrix:
    """The Robin subdomain operator of strip s (2-D): the global paper-form stencil on its
    columns with Dirichlet ghosts, plus the Robin diagonal terms on internal sides."""
    st = g.strips[s]
    lo, hi = robin_span(g, s)
    ax = g.alpha_outer(g.N_x, False)[lo:hi]
    axh = g.alpha_outer(g.N_x, True)[lo:hi + 1]
    A = assemble_5pt(ax, axh, g.alpha_outer(g.N_y, False), g.alpha_outer(g.N_y, True),
                     g.k2()[:, lo:hi], g.h).tolil()
    W = hi - lo
    ih2 = 1.0 / (g.h * g.h)
    if st.left_pad:                      # internal left side: Robin at lo - 1/2
        rho = robin_rho(g, lo)
        for l in range(g.N_y):
            A[l * W, l * W] += -ax[0] * axh[0] * rho[l] * ih2
    if st.right_pad:                     # internal right side: Robin at hi - 1/2
        rho = robin_rho(g, hi - 1)
        for l in range(g.N_y):
            A[l * W + W - 1, l * W + W - 1] += -ax[W - 1] * axh[W] * rho[l] * ih2
    return A.tocsr()


class RobinSolvers:
    """SuperLU factorisations of the Robin subdomain operators."""

    def __init__(self, g: Geometry):
        if g.dim != 2:
            raise ValueError("the Robin double sweep is built for 2-D problems")
        self.g = g
        self.lu = [spla.splu(assemble_robin_strip(g, s).tocsc(), permc_spec="COLAMD")
                   for s in range(g.J)]

    def solve(self, s: int, rhs: np.ndarray) -> np.ndarray:
        return self.lu[s].solve(rhs.ravel().astype(np.complex128)).reshape(rhs.shape)


def sweep_robin(g: Geometry, R: RobinSolvers, A, f: np.ndarray):
    """Right sweep on f, residual, left sweep on the residual; returns (v, w, g)."""
    J, h = g.J, g.h
    ih2 = 1.0 / (h * h)
    v = np.zeros_like(f)
    prev = None
    for s in range(J):
        lo, hi = robin_span(g, s)
        st = g.strips[s]
        rhs = np.zeros((g.N_y, hi - lo), dtype=np.complex128)
        clo, chi = st.core
        rhs[:, clo - lo:chi - lo] = f[:, clo:chi]                       # f^(j) on D^(j)
        if prev is not None:
            plo, px = prev                                              # data of v^(j-1)
            rho = robin_rho(g, lo)
            vi = px[:, lo - plo]              # v^(j-1) at the column inside subdomain j
            vo = px[:, lo - 1 - plo]          # and at the column outside it
            rhs[:, 0] += (vo - rho * vi) * ih2
        x = R.solve(s, rhs)
        v[:, clo:chi] = x[:, clo - lo:chi - lo]
        prev = (lo, x)
    res = f - (A @ v.ravel()).reshape(f.shape)
    w = np.zeros_like(f)
    nxt = None
    for s in range(J - 1, -1, -1):
        lo, hi = robin_span(g, s)
        st = g.strips[s]
        rhs = np.zeros((g.N_y, hi - lo), dtype=np.complex128)
        klo, khi = st.keep_dn
        rhs[:, klo - lo:khi - lo] = res[:, klo:khi]                     # g^(j) on D~^(j)
        if nxt is not None:
            nlo, nx_ = nxt                                              # data of w^(j+1)
            rho = robin_rho(g, hi - 1)
            wi = nx_[:, hi - 1 - nlo]         # w^(j+1) at the column inside subdomain j
            wo = nx_[:, hi - nlo]             # and at the column outside it
            rhs[:, hi - 1 - lo] += (wo - rho * wi) * ih2
        x = R.solve(s, rhs)
        w[:, klo:khi] = x[:, klo - lo:khi - lo]
        nxt = (lo, x)
    return v, w, res


def apply_P_robin(g: Geometry, R: RobinSolvers, A, f: np.ndarray) -> np.ndarray:
    v, w, _ = sweep_robin(g, R, A, f)
    return v + w


def apply_P_concurrent_robin(g: Geometry, R: RobinSolvers, A, f: np.ndarray,
                             start=None) -> np.ndarray:
    """The concurrent sweeps of Sec. 3.1 with Robin transmission: the iterative method of
    Sec. 1 (every subdomain problem takes Robin data from both neighbours' previous
    solutions), in which step n = 1..J updates only subdomains n and J + 1 - n; the two
    chains meet in the middle, where each takes the other's data from the step before.
    Returns v = v^(j) on D^(j) after step J.  `start` (optional, for pins) gives every
    subdomain's solution before step 1 as a global field (default zero)."""
    J, h = g.J, g.h
    ih2 = 1.0 / (h * h)
    spans = [robin_span(g, s) for s in range(J)]
    if start is None:
        V = [None] * J                      # latest solution of every subdomain (its columns)
    else:
        V = [start[:, lo:hi].copy() for (lo, hi) in spans]

    def solve(s, Vold):
        lo, hi = spans[s]
        st = g.strips[s]
        clo, chi = st.core
        rhs = np.zeros((g.N_y, hi - lo), dtype=np.complex128)
        rhs[:, clo - lo:chi - lo] = f[:, clo:chi]
        if s > 0 and Vold[s - 1] is not None:           # left side: data of subdomain s - 1
            plo, _ = spans[s - 1]
            vi = Vold[s - 1][:, lo - plo]
            vo = Vold[s - 1][:, lo - 1 - plo]
            rhs[:, 0] += (vo - robin_rho(g, lo) * vi) * ih2
        if s < J - 1 and Vold[s + 1] is not None:       # right side: data of subdomain s + 1
            nlo, _ = spans[s + 1]
            wi = Vold[s + 1][:, hi - 1 - nlo]
            wo = Vold[s + 1][:, hi - nlo]
            rhs[:, hi - 1 - lo] += (wo - robin_rho(g, hi - 1) * wi) * ih2
        return R.solve(s, rhs)

    for n in range(1, J + 1):
        upd = sorted({n - 1, J - n})                    # 0-based subdomains n and J + 1 - n
        new = {s: solve(s, V) for s in upd}             # both from the previous step's values
        for s, x in new.items():
            V[s] = x
    v = np.zeros_like(f)
    for s in range(J):
        lo, _ = spans[s]
        clo, chi = g.strips[s].core
        v[:, clo:chi] = V[s][:, clo - lo:chi - lo]
    return v
