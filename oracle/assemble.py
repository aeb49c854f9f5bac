"""Finite-difference Helmholtz operator with PML (oracle).

The operator is the paper's (Sec. 2.2): the standard 5-point approximation of
-d_xx - d_yy - k^2, where inside a PML each second derivative d_x(d_x u) becomes
alpha_x(x_i) [alpha_x(x_{i+1/2}) (u_{i+1} - u_i) - alpha_x(x_{i-1/2}) (u_i - u_{i-1})] / h^2.
With alpha = 1 it is exactly the textbook 5-point stencil.  Rows are written in this
(paper) form; the matrix is therefore not symmetric, but D^{-1} A is, with
D = diag(alpha_x(x_i) alpha_y(y_l)).

Unknown (l, i) has flat index l * N_x + i.  Values beyond the last row/column are
homogeneous Dirichlet ghosts.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .grid import Geometry, StripGeom


def assemble_5pt(ax: np.ndarray, axh: np.ndarray, ay: np.ndarray, ayh: np.ndarray,
                 k2: np.ndarray, h: float) -> sp.csr_matrix:
    """Assemble the paper-form operator on an Ny x Nx grid.

    ax  : alpha_x at the Nx points,  axh : alpha_x at the Nx+1 half-points
          (axh[m] sits between points m-1 and m)
    ay, ayh : the same along y
    k2  : k^2 at the points, shape (Ny, Nx)
    """
    Ny, Nx = k2.shape
    assert ax.shape == (Nx,) and axh.shape == (Nx + 1,)
    assert ay.shape == (Ny,) and ayh.shape == (Ny + 1,)
    inv_h2 = 1.0 / (h * h)
    L, I = np.meshgrid(np.arange(Ny), np.arange(Nx), indexing="ij")
    p = (L * Nx + I).ravel()
    axI, ayL = ax[I].ravel(), ay[L].ravel()
    east = axh[I + 1].ravel()     # alpha_x(x_{i+1/2})
    west = axh[I].ravel()         # alpha_x(x_{i-1/2})
    north = ayh[L + 1].ravel()    # alpha_y(y_{l+1/2})
    south = ayh[L].ravel()        # alpha_y(y_{l-1/2})
    Iv, Lv = I.ravel(), L.ravel()

    rows, cols, vals = [], [], []
    # diagonal
    rows.append(p); cols.append(p)
    vals.append(axI * (east + west) * inv_h2 + ayL * (north + south) * inv_h2 - k2.ravel())
    # x neighbours
    m = Iv + 1 < Nx
    rows.append(p[m]); cols.append(p[m] + 1); vals.append(-axI[m] * east[m] * inv_h2)
    m = Iv - 1 >= 0
    rows.append(p[m]); cols.append(p[m] - 1); vals.append(-axI[m] * west[m] * inv_h2)
    # y neighbours
    m = Lv + 1 < Ny
    rows.append(p[m]); cols.append(p[m] + Nx); vals.append(-ayL[m] * north[m] * inv_h2)
    m = Lv - 1 >= 0
    rows.append(p[m]); cols.append(p[m] - Nx); vals.append(-ayL[m] * south[m] * inv_h2)

    A = sp.coo_matrix((np.concatenate(vals).astype(np.complex128),
                       (np.concatenate(rows), np.concatenate(cols))), shape=(Ny * Nx, Ny * Nx))
    return A.tocsr()


def assemble_7pt(ax: np.ndarray, axh: np.ndarray, ay: np.ndarray, ayh: np.ndarray,
                 az: np.ndarray, azh: np.ndarray, k2: np.ndarray, h: float) -> sp.csr_matrix:
    """The 3-D paper-form operator (Sec. 2.2: the same second-difference form along each
    of x, y, z) on an Nz x Ny x Nx grid; unknown (z, l, i) has flat index
    (z * Ny + l) * Nx + i.  Tables as in assemble_5pt, az/azh along z; k2 (Nz, Ny, Nx)."""
    Nz, Ny, Nx = k2.shape
    assert ax.shape == (Nx,) and axh.shape == (Nx + 1,)
    assert ay.shape == (Ny,) and ayh.shape == (Ny + 1,)
    assert az.shape == (Nz,) and azh.shape == (Nz + 1,)
    inv_h2 = 1.0 / (h * h)
    Z, L, I = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    Z, L, I = Z.ravel(), L.ravel(), I.ravel()
    p = (Z * Ny + L) * Nx + I
    rows, cols, vals = [p], [p], []
    diag = -k2.ravel().astype(np.complex128)
    # one axis at a time: alpha(point) [alpha(+half)(u+ - u) - alpha(-half)(u - u-)] / h^2
    for idx, n, a, ah, stride in ((I, Nx, ax, axh, 1), (L, Ny, ay, ayh, Nx), (Z, Nz, az, azh, Nx * Ny)):
        ap, plus, minus = a[idx], ah[idx + 1], ah[idx]
        diag = diag + ap * (plus + minus) * inv_h2
        m = idx + 1 < n
        rows.append(p[m]); cols.append(p[m] + stride); vals.append(-ap[m] * plus[m] * inv_h2)
        m = idx - 1 >= 0
        rows.append(p[m]); cols.append(p[m] - stride); vals.append(-ap[m] * minus[m] * inv_h2)
    vals.insert(0, diag)
    A = sp.coo_matrix((np.concatenate(vals).astype(np.complex128),
                       (np.concatenate(rows), np.concatenate(cols))), shape=(p.size, p.size))
    return A.tocsr()


def assemble_global(g: Geometry) -> sp.csr_matrix:
    """The global operator A on the padded grid."""
    if g.dim == 3:
        return assemble_7pt(g.alpha_outer(g.N_x, False), g.alpha_outer(g.N_x, True),
                            g.alpha_outer(g.N_y, False), g.alpha_outer(g.N_y, True),
                            g.alpha_outer(g.N_z, False), g.alpha_outer(g.N_z, True),
                            g.k2(), g.h)
    return assemble_5pt(g.alpha_outer(g.N_x, False), g.alpha_outer(g.N_x, True),
                        g.alpha_outer(g.N_y, False), g.alpha_outer(g.N_y, True),
                        g.k2(), g.h)


def assemble_strip(g: Geometry, st: StripGeom, k2=None) -> sp.csr_matrix:
    """The padded strip operator A^(j) (Sec. 2.1-2.2, grid of eq. grid_A_j): its own
    x-PML pads on internal sides, the global y-PML (and z-PML in 3-D), the medium continued
    into the pads."""
    if g.dim == 3:
        return assemble_7pt(g.alpha_strip_x(st, False), g.alpha_strip_x(st, True),
                            g.alpha_outer(g.N_y, False), g.alpha_outer(g.N_y, True),
                            g.alpha_outer(g.N_z, False), g.alpha_outer(g.N_z, True),
                            g.strip_k2(st, k2), g.h)
    return assemble_5pt(g.alpha_strip_x(st, False), g.alpha_strip_x(st, True),
                        g.alpha_outer(g.N_y, False), g.alpha_outer(g.N_y, True),
                        g.strip_k2(st, k2), g.h)


def apply_A(A: sp.csr_matrix, u: np.ndarray) -> np.ndarray:
    """A u for a field u of shape (N_y, N_x)."""
    return (A @ u.ravel()).reshape(u.shape)


def pml_scaling(g: Geometry) -> np.ndarray:
    """D = alpha_x(x_i) alpha_y(y_l) (alpha_z(z) in 3-D) on the padded grid: A = D S with S
    complex symmetric."""
    ax = g.alpha_outer(g.N_x, False)
    ay = g.alpha_outer(g.N_y, False)
    if g.dim == 3:
        az = g.alpha_outer(g.N_z, False)
        return az[:, None, None] * ay[None, :, None] * ax[None, None, :]
    return ay[:, None] * ax[None, :]
