"""The double-sweep domain-decomposition preconditioner P (oracle).

Written step by step after Sec. 2.1-2.3 of the paper:
  upward sweep   (eq. solve_upward):   A^(j) v^(j) = f^(j) - 2 delta(x - b_{j-1}) d_x v^(j-1)
  residual                              g = f - A v   on the whole grid
  downward sweep (eq. solve_downward): A~^(j) w^(j) = g^(j) + 2 delta(x - b~_j) d_x w^(j+1)
  P f = v + w
with the discrete derivative d_x u(x_{j+1/2}) = (u_{j+1} - u_j)/h and the discrete
delta equal to 1/(2h) on the two grid columns next to the half-point (Sec. 2.2).
The same padded strip operator serves both sweeps (Sec. 2.2: A~^(j) = A^(j) once the
second boundary set is beta~_j = beta_j + 1).

The reduced form (Sec. 2.3, Algorithms 2-4) keeps only the columns beta_j, beta_j+1
(0-based) of each internal interface.

Every subdomain solve is a SuperLU factorisation of the assembled strip matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import assemble_global, assemble_strip
from .grid import Geometry


class StripSolvers:
    """SuperLU factorisations of all padded strip operators A^(j) (Algorithm 1)."""

    def __init__(self, g: Geometry, k2=None, progress=None):
        """progress: optional callable(strips done, J), called after each factorisation."""
        self.g = g
        k2 = g.k2() if k2 is None else k2
        self.lu = []
        for st in g.strips:
            As = assemble_strip(g, st, k2).tocsc()
            self.lu.append(spla.splu(As, permc_spec="COLAMD"))
            if progress is not None:
                progress(len(self.lu), g.J)

    def solve(self, s: int, rhs: np.ndarray) -> np.ndarray:
        st = self.g.strips[s]
        assert rhs.shape == self.g.strip_shape(st)
        return self.lu[s].solve(rhs.ravel().astype(np.complex128)).reshape(rhs.shape)


def sweep(g: Geometry, S: StripSolvers, A, f: np.ndarray, up_from: int = 0, dn_from: int = None):
    """Both sweeps for input f (N_y, N_x), or (N_z, N_y, N_x) in 3-D (slabs along x, the
    transmission sources on two x-planes).  Returns (v, w, residual g).

    up_from / dn_from: first strip of each sweep (0-based).  The full preconditioner
    starts at strip 0 and at strip J-1; Algorithms 3 and 4 start at strip 1 and J-2
    because their inputs vanish on the skipped subdomains."""
    J, h = g.J, g.h
    if dn_from is None:
        dn_from = J - 1

    # ---- upward sweep, eq. solve_upward
    v = np.zeros_like(f)
    prev = None
    for s in range(up_from, J):
        st = g.strips[s]
        rhs = np.zeros(g.strip_shape(st), dtype=np.complex128)
        lo, hi = st.core
        rhs[..., lo - st.a:hi - st.a] = f[..., lo:hi]               # f^(j): f restricted to D^(j)
        if prev is not None:
            b = g.beta[s]                                          # b_{j-1} between columns b-1 and b
            pst, px = prev
            dxv = (px[..., b - pst.a] - px[..., b - 1 - pst.a]) / h   # d_x v^(j-1)(b_{j-1})
            delta = 1.0 / (2.0 * h)                                # discrete delta on columns b-1, b
            rhs[..., b - 1 - st.a] += -2.0 * delta * dxv
            rhs[..., b - st.a] += -2.0 * delta * dxv
        x = S.solve(s, rhs)
        v[..., lo:hi] = x[..., lo - st.a:hi - st.a]                   # v = v^(j) on D^(j)
        prev = (st, x)

    # ---- residual on the whole grid
    res = f - (A @ v.ravel()).reshape(f.shape)

    # ---- downward sweep, eq. solve_downward
    w = np.zeros_like(f)
    nxt = None
    for s in range(dn_from, -1, -1):
        st = g.strips[s]
        rhs = np.zeros(g.strip_shape(st), dtype=np.complex128)
        lo, hi = st.keep_dn
        rhs[..., lo - st.a:hi - st.a] = res[..., lo:hi]             # g^(j): g restricted to D~^(j)
        if nxt is not None:
            b = g.beta[s + 1]                                      # b~_j between columns b and b+1
            nst, nx_ = nxt
            dxw = (nx_[..., b + 1 - nst.a] - nx_[..., b - nst.a]) / h  # d_x w^(j+1)(b~_j)
            delta = 1.0 / (2.0 * h)
            rhs[..., b - st.a] += 2.0 * delta * dxw
            rhs[..., b + 1 - st.a] += 2.0 * delta * dxw
        x = S.solve(s, rhs)
        w[..., lo:hi] = x[..., lo - st.a:hi - st.a]                   # w = w^(j) on D~^(j)
        nxt = (st, x)
    return v, w, res


def apply_P(g: Geometry, S: StripSolvers, A, f: np.ndarray) -> np.ndarray:
    """P f = v + w (Sec. 2.1, end)."""
    v, w, _ = sweep(g, S, A, f)
    return v + w


def apply_AP_full(g: Geometry, S: StripSolvers, A, f: np.ndarray) -> np.ndarray:
    pf = apply_P(g, S, A, f)
    return (A @ pf.ravel()).reshape(f.shape)


# ------------------------------------------------------------------ reduced form

def reduced_setup(g: Geometry, S: StripSolvers, A, f: np.ndarray):
    """Algorithm 2: u~^(j) = A^(j)^{-1} f~^(j) with f~^(j) = f on D~^(j); u~ = u~^(j) on
    D~^(j); returns (u~, phi = f - A u~)."""
    ut = np.zeros_like(f)
    for s, st in enumerate(g.strips):
        rhs = np.zeros(g.strip_shape(st), dtype=np.complex128)
        lo, hi = st.keep_dn
        rhs[..., lo - st.a:hi - st.a] = f[..., lo:hi]
        x = S.solve(s, rhs)
        ut[..., lo:hi] = x[..., lo - st.a:hi - st.a]
    phi = f - (A @ ut.ravel()).reshape(f.shape)
    return ut, phi


def to_reduced(g: Geometry, field: np.ndarray) -> np.ndarray:
    """Restriction of a field to the reduced columns, shape (N_y, 2(J-1)) (3-D: the reduced
    planes, (N_z, N_y, 2(J-1)))."""
    return field[..., g.reduced_columns()].copy()


def from_reduced(g: Geometry, red: np.ndarray) -> np.ndarray:
    out = np.zeros(g.field_shape, dtype=np.complex128)
    out[..., g.reduced_columns()] = red
    return out


def apply_AP_reduced(g: Geometry, S: StripSolvers, A, psi_red: np.ndarray) -> np.ndarray:
    """Algorithm 3 on a reduced vector: upward sweep j = 2..J, g = psi - A v, downward
    sweep j = J-1..1, h = g - A w, output psi - h (restricted to the reduced columns)."""
    psi = from_reduced(g, psi_red)
    v, w, res = sweep(g, S, A, psi, up_from=1, dn_from=g.J - 2)
    hres = res - (A @ w.ravel()).reshape(psi.shape)
    return to_reduced(g, psi - hres)


def apply_P_reduced(g: Geometry, S: StripSolvers, A, psi_red: np.ndarray, ut: np.ndarray) -> np.ndarray:
    """Algorithm 4: v + w for input psi (sweeps as in Algorithm 3), plus u~."""
    psi = from_reduced(g, psi_red)
    v, w, _ = sweep(g, S, A, psi, up_from=1, dn_from=g.J - 2)
    return v + w + ut


# ------------------------------------------------------------------ concurrent double sweep
#
# The paper observes (Sec. 1 and the end of Sec. 3.1) that the upward and downward sequences
# of solves can run at the same time if the point where they cross is handled with care; it
# shows this only for its 1-D model.  The 2-D form used here needs no crossing point at all:
#   upward  (as in eq. solve_upward)          v^(j)  = A^(j)^{-1}(f^(j)  - 2 delta(x - b_{j-1}) d_x v^(j-1))
#   downward on f instead of the residual     w'^(j) = A^(j)^{-1}(f~^(j) + 2 delta(x - b~_j) d_x w'^(j+1))
#   the strip's own sources, in both          z^(j)  = A^(j)^{-1}(f on D^(j) and D~^(j))
#   P_c f = v^(j) + w'^(j) - z^(j) on D^(j)
# v^(j) carries the field of every source left of b_j, w'^(j) that of every source right of
# b_{j-1} (the transmission reproduces the incoming wave, Sec. 3.2), so their sum counts the
# sources of D^(j) and D~^(j) twice and z^(j) removes one copy.  For a medium independent of x
# and perfect PML layers P_c f is the solution (the argument of Theorem 1 in each direction).
# The two chains do not depend on each other, and the z^(j) on nothing.

def sweep_concurrent(g: Geometry, S: StripSolvers, f: np.ndarray):
    """Both sweeps of the concurrent form on f; returns (v, w', z) on the whole grid, each
    restricted to the columns of D^(j) of its strip j."""
    J, h = g.J, g.h
    delta = 1.0 / (2.0 * h)
    v = np.zeros_like(f)
    wd = np.zeros_like(f)
    z = np.zeros_like(f)
    prev = None
    for s in range(J):                                   # upward, as in sweep()
        st = g.strips[s]
        rhs = np.zeros(g.strip_shape(st), dtype=np.complex128)
        lo, hi = st.core
        rhs[..., lo - st.a:hi - st.a] = f[..., lo:hi]
        if prev is not None:
            b = g.beta[s]
            pst, px = prev
            dxv = (px[..., b - pst.a] - px[..., b - 1 - pst.a]) / h
            rhs[..., b - 1 - st.a] += -2.0 * delta * dxv
            rhs[..., b - st.a] += -2.0 * delta * dxv
        x = S.solve(s, rhs)
        v[..., lo:hi] = x[..., lo - st.a:hi - st.a]
        prev = (st, x)
    nxt = None
    for s in range(J - 1, -1, -1):                       # downward on f
        st = g.strips[s]
        rhs = np.zeros(g.strip_shape(st), dtype=np.complex128)
        lo, hi = st.keep_dn
        rhs[..., lo - st.a:hi - st.a] = f[..., lo:hi]        # f~^(j): f on D~^(j)
        if nxt is not None:
            b = g.beta[s + 1]
            nst, nx_ = nxt
            dxw = (nx_[..., b + 1 - nst.a] - nx_[..., b - nst.a]) / h
            rhs[..., b - st.a] += 2.0 * delta * dxw
            rhs[..., b + 1 - st.a] += 2.0 * delta * dxw
        x = S.solve(s, rhs)
        clo, chi = st.core
        wd[..., clo:chi] = x[..., clo - st.a:chi - st.a]
        nxt = (st, x)
    for s, st in enumerate(g.strips):                    # the strips' own sources
        rhs = np.zeros(g.strip_shape(st), dtype=np.complex128)
        lo, hi = max(st.core[0], st.keep_dn[0]), min(st.core[1], st.keep_dn[1])
        rhs[..., lo - st.a:hi - st.a] = f[..., lo:hi]
        x = S.solve(s, rhs)
        clo, chi = st.core
        z[..., clo:chi] = x[..., clo - st.a:chi - st.a]
    return v, wd, z


def apply_P_concurrent(g: Geometry, S: StripSolvers, f: np.ndarray) -> np.ndarray:
    """P_c f = v + w' - z (the concurrent double sweep)."""
    v, wd, z = sweep_concurrent(g, S, f)
    return v + wd - z


def concurrent_columns(g: Geometry) -> np.ndarray:
    """Columns where f - A P_c f can be non-zero: beta_j - 1 and beta_j of every internal
    interface (the two columns next to b_j)."""
    return g.residual_columns()


def reduced_setup_concurrent(g: Geometry, S: StripSolvers, A, f: np.ndarray):
    """The reduced form's starting point for P_c: u~ from independent strip solves of f on
    D^(j), kept on D^(j); phi = f - A u~ then lives on the concurrent columns."""
    ut = np.zeros_like(f)
    for s, st in enumerate(g.strips):
        rhs = np.zeros(g.strip_shape(st), dtype=np.complex128)
        lo, hi = st.core
        rhs[..., lo - st.a:hi - st.a] = f[..., lo:hi]
        x = S.solve(s, rhs)
        ut[..., lo:hi] = x[..., lo - st.a:hi - st.a]
    phi = f - (A @ ut.ravel()).reshape(f.shape)
    return ut, phi


def apply_AP_concurrent_reduced(g: Geometry, S: StripSolvers, A, psi_red: np.ndarray) -> np.ndarray:
    """(A P_c psi) restricted to the concurrent columns, for psi given there."""
    cols = concurrent_columns(g)
    psi = np.zeros(g.field_shape, dtype=np.complex128)
    psi[..., cols] = psi_red
    out = (A @ apply_P_concurrent(g, S, psi).ravel()).reshape(psi.shape)
    return out[..., cols].copy()
