"""Padded grid, subdomain partition and PML coefficient tables (oracle).

Conventions (0-based; the paper counts from 1):
  * The discrete unknowns live on the padded grid of N_x x N_y points, N = n + 2 w_out:
    the n_x x n_y interior of the unit square (Sec. 2.2, grid spacing h in x and y) plus
    an outer PML of w_out points on every face.  Columns are x (index i), rows are y
    (index l).  Homogeneous Dirichlet values sit at the ghost points just outside.
  * The PML replaces d/dx by alpha_x d/dx with alpha = 1/(1 + i sigma/omega)
    (Sec. 2.1); sigma vanishes in the interior and grows inside the layer.  The
    paper gives no profile; the reading used here is sigma(xi) = sigma_max
    (xi/(w h))^p with depth xi measured from the layer's inner edge, the edge at a
    half-point, layer points at xi = (m - 1/2) h and half-points at xi = m h, and
    sigma_max = s0 c_ref / (w h) with c_ref the largest wave speed.  The outer PML
    (which belongs to the global operator A and so to the solution) and the interface
    pads (which belong only to the strip operators A^(j), i.e. to the preconditioner)
    take their own strengths: s0 and s0_iface.  Unless given, s0_iface = 2.5 w: the pads
    then have the same damping per cell whatever their width, sigma_max h / c_ref = 2.5
    (chosen with this oracle on the constant-medium study of Table 4, Sec. 4.4).
  * Strips (Sec. 2.2): interfaces at half-points.  beta[0] = 0, beta[J] = N_x and, for
    0 < s < J, strip s-1 ends at column beta[s]-1 and strip s starts at column beta[s]
    (the paper's b_j = x_{beta_j + 1/2} in 1-based counting).  Core of strip s (0-based
    s = 0..J-1): columns [beta[s], beta[s+1]).
  * The operator A^(j) of a strip covers its core plus one extra column on the right
    (the shifted boundary beta~_j = beta_j + 1, Sec. 2.2) and is padded with w PML
    columns on each internal side.
  * Default partition: the interior is split evenly, beta[s] = w_out + floor(s n_x / J + 1/2);
    rule "paper" follows eq. define_beta_j, beta_j ~ w + j (N_x - 2w - 1)/J.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


# interface pads: sigma_max h / c_ref unless their strength is given
PAD_S0_PER_CELL = 2.5


def _sigma(depth_cells: np.ndarray, width: int, h: float, sigma_max: float, power: float) -> np.ndarray:
    """sigma at depth xi = depth_cells * h inside a layer of `width` cells."""
    d = np.clip(depth_cells, 0.0, None)
    if width <= 0:
        return np.zeros_like(d)
    return sigma_max * (d / width) ** power


def _alpha(sigma: np.ndarray, omega: float) -> np.ndarray:
    """Complex stretching factor alpha = 1 / (1 + i sigma / omega) (Sec. 2.1)."""
    return 1.0 / (1.0 + 1j * sigma / omega)


@dataclass
class StripGeom:
    s: int          # 0-based strip index
    a: int          # first global column of the padded strip domain
    W: int          # number of columns of the padded strip domain
    core: tuple     # [lo, hi) global core columns  (D^(j))
    dom: tuple      # [lo, hi) global non-pad columns (core plus the extra column)
    keep_dn: tuple  # [lo, hi) global columns of D~^(j) (downward sweep keeps these)
    left_pad: bool
    right_pad: bool

    def local(self, col: int) -> int:
        return col - self.a


@dataclass
class Geometry:
    n_x: int
    n_y: int
    w_out: int
    w: int
    J: int
    h: float
    omega: float
    c: np.ndarray                  # interior wave speed (n_y, n_x)
    power: float = 2.0
    s0: float = 10.0
    beta: np.ndarray = None        # length J+1
    strips: List[StripGeom] = field(default_factory=list)
    cref: Optional[float] = None   # PML reference speed; None -> max(c)
    s0_iface: Optional[float] = None  # strength of the interface pads (strip operators
                                      # only); None: PAD_S0_PER_CELL * w
    n_z: int = 0                   # 3-D (Sec. 2.2, 7-point stencil): interior points along z;
                                   # 0 for the 2-D problem.  c is then (n_z, n_y, n_x)

    @property
    def dim(self) -> int:
        return 3 if self.n_z else 2

    @property
    def N_z(self) -> int:
        return self.n_z + 2 * self.w_out if self.n_z else 1

    @property
    def field_shape(self) -> tuple:
        """Shape of a field on the padded grid: (N_y, N_x), or (N_z, N_y, N_x) in 3-D."""
        return (self.N_z, self.N_y, self.N_x) if self.n_z else (self.N_y, self.N_x)

    def strip_shape(self, st: "StripGeom") -> tuple:
        return self.field_shape[:-1] + (st.W,)

    @property
    def N_x(self) -> int:
        return self.n_x + 2 * self.w_out

    @property
    def N_y(self) -> int:
        return self.n_y + 2 * self.w_out

    @property
    def c_ref(self) -> float:
        return float(np.max(self.c)) if self.cref is None else float(self.cref)

    # ---------------------------------------------------------------- medium
    def k2(self) -> np.ndarray:
        """k^2 = omega^2 / c^2 on the padded grid, the medium continued into the outer
        PML by its value on the nearest interior point."""
        cp = np.pad(self.c, self.w_out, mode="edge")
        return (self.omega / cp) ** 2

    def clamp_index(self):
        """For every padded point, the flat interior index it takes its medium from."""
        Ny, Nx = self.N_y, self.N_x
        li = np.clip(np.arange(Ny) - self.w_out, 0, self.n_y - 1)
        ii = np.clip(np.arange(Nx) - self.w_out, 0, self.n_x - 1)
        if self.n_z:
            zi = np.clip(np.arange(self.N_z) - self.w_out, 0, self.n_z - 1)
            return ((zi[:, None, None] * self.n_y + li[None, :, None]) * self.n_x + ii[None, None, :])
        return (li[:, None] * self.n_x + ii[None, :])

    # ---------------------------------------------------------------- PML tables
    @property
    def s0_pad(self) -> float:
        """Strength s0 of the interface pads."""
        return PAD_S0_PER_CELL * self.w if self.s0_iface is None else float(self.s0_iface)

    def sigma_max(self, width: int, s0: Optional[float] = None) -> float:
        s0 = self.s0 if s0 is None else s0
        return s0 * self.c_ref / (width * self.h) if width > 0 else 0.0

    def outer_depth(self, pos: np.ndarray, N: int) -> np.ndarray:
        """Depth (in cells) of position `pos` (points integer, half-points x.5) inside the
        outer PML of an axis with N points."""
        lo_edge = self.w_out - 0.5
        hi_edge = N - self.w_out - 0.5
        return np.maximum(np.maximum(lo_edge - pos, pos - hi_edge), 0.0)

    def alpha_outer(self, N: int, half: bool) -> np.ndarray:
        """alpha along an axis of N points: at the points 0..N-1, or (half=True) at the
        N+1 half-points, entry m being the half-point between points m-1 and m."""
        pos = np.arange(N + 1) - 0.5 if half else np.arange(N, dtype=float)
        sig = _sigma(self.outer_depth(pos, N), self.w_out, self.h, self.sigma_max(self.w_out), self.power)
        return _alpha(sig, self.omega)

    def alpha_strip_x(self, st: StripGeom, half: bool) -> np.ndarray:
        """alpha_x of the padded operator A^(j) of strip `st`, at its W points or W+1
        half-points (strip-local indexing as in alpha_outer)."""
        if half:
            pos = st.a + np.arange(st.W + 1) - 0.5
        else:
            pos = st.a + np.arange(st.W, dtype=float)
        depth_out = self.outer_depth(pos, self.N_x)
        sig = _sigma(depth_out, self.w_out, self.h, self.sigma_max(self.w_out), self.power)
        smax_pad = self.sigma_max(self.w, self.s0_pad)
        if st.left_pad:
            edge = st.core[0] - 0.5
            m = pos < edge
            sig = np.where(m, _sigma(edge - pos, self.w, self.h, smax_pad, self.power), sig)
        if st.right_pad:
            edge = st.dom[1] - 0.5
            m = pos > edge
            sig = np.where(m, _sigma(pos - edge, self.w, self.h, smax_pad, self.power), sig)
        return _alpha(sig, self.omega)

    def strip_k2(self, st: StripGeom, k2: Optional[np.ndarray] = None) -> np.ndarray:
        """Medium of A^(j) on the strip (N_y, W) (3-D: (N_z, N_y, W)): the true k^2 on the
        non-pad columns and, in each pad, k^2 of the adjacent non-pad column (x-independent
        extension, Sec. 2.1)."""
        if k2 is None:
            k2 = self.k2()
        cols = st.a + np.arange(st.W)
        cols = np.clip(cols, st.dom[0], st.dom[1] - 1)
        return k2[..., cols]

    # ---------------------------------------------------------------- index sets
    def reduced_columns(self) -> np.ndarray:
        """Columns carrying the reduced unknowns: beta_j and beta_j + 1 for each internal
        interface (the paper's beta_j+1, beta_j+2 in 1-based counting, Sec. 2.3)."""
        out = []
        for s in range(1, self.J):
            out += [self.beta[s], self.beta[s] + 1]
        return np.array(out, dtype=int)

    def residual_columns(self) -> np.ndarray:
        """Columns where f - A v can be non-zero after the upward sweep: beta_j - 1, beta_j."""
        out = []
        for s in range(1, self.J):
            out += [self.beta[s] - 1, self.beta[s]]
        return np.array(out, dtype=int)


def partition(n_x: int, w_out: int, J: int, w: int, rule: str = "interior") -> np.ndarray:
    N_x = n_x + 2 * w_out
    b = np.zeros(J + 1, dtype=int)
    b[J] = N_x
    for s in range(1, J):
        if rule == "interior":
            b[s] = w_out + int(math.floor(s * n_x / J + 0.5))
        elif rule == "paper":
            b[s] = int(math.floor(w + s * (N_x - 2 * w - 1) / J + 0.5))
        else:
            raise ValueError(rule)
    return b


def make_geometry(c: np.ndarray, omega: float, h: float, w_out: int, w: int, J: int,
                  power: float = 2.0, s0: float = 10.0, beta: Optional[Sequence[int]] = None,
                  rule: str = "interior", cref: Optional[float] = None,
                  s0_iface: Optional[float] = None) -> Geometry:
    c = np.asarray(c, dtype=float)
    n_z = 0
    if c.ndim == 3:
        n_z, n_y, n_x = c.shape       # 3-D: slabs along x (Sec. 2.2, 3-D case)
    else:
        n_y, n_x = c.shape
    if J < 1:
        raise ValueError("J must be >= 1")
    if beta is None:
        b = partition(n_x, w_out, J, w, rule)
    else:
        b = np.concatenate([[0], np.asarray(beta, dtype=int), [n_x + 2 * w_out]])
        if len(b) != J + 1:
            raise ValueError("beta must list J-1 interfaces")
    N_x = n_x + 2 * w_out
    for s in range(1, J + 1):
        if b[s] - b[s - 1] < 2:
            raise ValueError("every strip core needs at least two columns")
    for s in range(1, J):
        if b[s] - 1 < w_out or b[s] + 1 > w_out + n_x - 1:
            raise ValueError("interfaces must lie inside the interior (outside the outer PML)")
    g = Geometry(n_x, n_y, w_out, w, J, h, omega, c, power, s0, b, cref=cref, n_z=n_z,
                 s0_iface=s0_iface)
    for s in range(J):
        lp = s > 0
        rp = s < J - 1
        core = (int(b[s]), int(b[s + 1]))
        dom = (core[0], core[1] + (1 if rp else 0))
        a = core[0] - (w if lp else 0)
        W = (dom[1] + (w if rp else 0)) - a
        keep_dn = (core[0] + (1 if lp else 0), core[1] + (1 if rp else 0))
        g.strips.append(StripGeom(s, a, W, core, dom, keep_dn, lp, rp))
    return g


def geometry_from_workload(wl) -> Geometry:
    return make_geometry(wl.c, wl.omega, wl.h, wl.w_out, wl.w, wl.J, wl.pml_power, wl.pml_s0,
                         wl.beta, s0_iface=wl.pml_iface_s0)
