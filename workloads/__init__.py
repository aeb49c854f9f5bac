"""Seeded synthetic inputs for the PML-transmission double-sweep Helmholtz solver.

This module only produces *inputs*: wave-speed fields, source positions, right-hand
sides and the numeric parameters of each workload.  It contains none of the
method's arithmetic (no operator, no PML coefficients, no solves), so both the
CPU oracle tests and the GPU path may use it without sharing any of the method.

Workloads follow the paper's setting (unit square, 10 points per wavelength,
residual reduction 1e-6; Sections 4.1-4.4) with seeded synthetic media standing
in for the paper's datasets (the Marmousi model and the random media are not
available).  Grid coordinates: interior point (i, l), 0-based, sits at
(i*h, l*h); fields on the padded grid are arrays of shape (N_y, N_x) with x
fastest (C order).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

__all__ = [
    "Workload", "homogeneous_100", "lens_1000", "layers", "layers_uneven_batch", "smooth_500", "small",
    "smoothed_noise", "point_sources", "padded_rhs", "WORKLOADS", "small3", "smooth_3d",
]


@dataclass
class Workload:
    """One solver workload: medium, frequency, discretisation and sources.

    c        : interior wave speed, shape (n_y, n_x), float64
    omega    : angular frequency
    h        : grid spacing (equal in x and y)
    w_out    : outer PML width in cells (all four faces)
    w        : interface PML width in cells (pads on internal strip sides)
    J        : number of strips along x
    src      : list of (i, l) interior source indices; f = 1/h^2 at each
    pml_power, pml_s0 : PML profile sigma(xi) = sigma_max (xi/(w h))^p with
               sigma_max = s0 c_ref / (w h); p = pml_power, s0 = pml_s0 (outer PML)
    pml_iface_s0 : s0 of the interface pads (they enter only the strip operators);
               None: the library's default, 2.5 times the pad width
    """
    name: str
    c: np.ndarray
    omega: float
    h: float
    w_out: int
    w: int
    J: int
    src: List[tuple]
    pml_power: float = 2.0
    pml_s0: float = 10.0
    tol: float = 1e-6
    pml_iface_s0: Optional[float] = None
    precision: str = "c128"
    beta: Optional[List[int]] = None
    extra: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return int(self.c.ndim)

    @property
    def n_x(self) -> int:
        return int(self.c.shape[-1])

    @property
    def n_y(self) -> int:
        return int(self.c.shape[-2])

    @property
    def n_z(self) -> int:
        """Interior points along z in 3-D (c of shape (n_z, n_y, n_x)); 0 in 2-D."""
        return int(self.c.shape[0]) if self.c.ndim == 3 else 0

    @property
    def N_z(self) -> int:
        return self.n_z + 2 * self.w_out if self.c.ndim == 3 else 1

    @property
    def n_points(self) -> int:
        """Interior grid points."""
        return int(self.c.size)

    @property
    def N_x(self) -> int:
        return self.n_x + 2 * self.w_out

    @property
    def N_y(self) -> int:
        return self.n_y + 2 * self.w_out

    @property
    def nrhs(self) -> int:
        return len(self.src)

    def rhs(self, which=None) -> np.ndarray:
        """Right-hand sides on the padded grid, shape (nrhs, N_y, N_x) complex128
        ((nrhs, N_z, N_y, N_x) in 3-D)."""
        return padded_rhs(self, which)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def padded_rhs(wl: Workload, which=None) -> np.ndarray:
    """Point sources of strength 1/h^2 (2-D) or 1/h^3 (3-D) on the padded grid."""
    srcs = wl.src if which is None else [wl.src[k] for k in which]
    if wl.dim == 3:
        f = np.zeros((len(srcs), wl.N_z, wl.N_y, wl.N_x), dtype=np.complex128)
        for k, (i, l, z) in enumerate(srcs):
            f[k, z + wl.w_out, l + wl.w_out, i + wl.w_out] = 1.0 / wl.h ** 3
        return f
    f = np.zeros((len(srcs), wl.N_y, wl.N_x), dtype=np.complex128)
    for k, (i, l) in enumerate(srcs):
        f[k, l + wl.w_out, i + wl.w_out] = 1.0 / wl.h ** 2
    return f


def smoothed_noise(shape, sigma_pts: float, seed: int) -> np.ndarray:
    """Unit-variance Gaussian white noise smoothed by a Gaussian of width sigma_pts grid
    points (periodic FFT filter), rescaled to zero mean and unit standard deviation."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape)
    ks = [np.fft.fftfreq(n) for n in shape]
    grids = np.meshgrid(*ks, indexing="ij")
    k2 = sum(g ** 2 for g in grids)
    filt = np.exp(-2.0 * (math.pi ** 2) * (sigma_pts ** 2) * k2)
    s = np.real(np.fft.ifftn(np.fft.fftn(z) * filt))
    s -= s.mean()
    sd = s.std()
    return s / sd if sd > 0 else s


def point_sources(n_x: int, n_y: int, count: int, seed: int, margin: int = 0) -> List[tuple]:
    """`count` distinct uniform-random interior points (i, l)."""
    rng = np.random.default_rng(seed)
    seen = set()
    out = []
    while len(out) < count:
        i = int(rng.integers(margin, n_x - margin))
        l = int(rng.integers(margin, n_y - margin))
        if (i, l) not in seen:
            seen.add((i, l))
            out.append((i, l))
    return out


def _layers_1d(n: int, seed: int, c_lo=1.5, c_hi=4.0, nl_lo=10, nl_hi=30) -> np.ndarray:
    rng = np.random.default_rng(seed)
    L = int(rng.integers(nl_lo, nl_hi + 1))
    cuts = np.sort(rng.uniform(0.0, 1.0, L - 1))
    vals = rng.uniform(c_lo, c_hi, L)
    y = np.arange(n) / n
    idx = np.searchsorted(cuts, y, side="right")
    return vals[idx]


# --------------------------------------------------------------------------- configs

def small(n=24, J=3, w_out=6, w=5, c=None, nsrc=1, seed=11, ppw=10.0, **kw) -> Workload:
    """Small homogeneous (or given) medium for oracle-sized parity tests."""
    h = 1.0 / n
    if c is None:
        c = np.ones((n, n))
    omega = 2 * math.pi / (ppw * h) * float(np.min(c))
    srcs = point_sources(c.shape[1], c.shape[0], nsrc, seed, margin=min(2, n // 4))
    return Workload(f"small{n}", np.asarray(c, float), omega, h, w_out, w, J, srcs, **kw)


def small3(n=10, J=2, w_out=4, w=3, c=None, nsrc=1, seed=13, ppw=8.0, **kw) -> Workload:
    """Small 3-D cube (n^3 interior) for oracle-sized parity tests; c (n, n, n) or 1."""
    h = 1.0 / n
    if c is None:
        c = np.ones((n, n, n))
    c = np.asarray(c, float)
    omega = 2 * math.pi / (ppw * h) * float(np.min(c))
    rng = np.random.default_rng(seed)
    m = min(2, n // 4)
    srcs = []
    while len(srcs) < nsrc:
        p = tuple(int(v) for v in rng.integers(m, n - m, 3))
        if p not in srcs:
            srcs.append(p)
    return Workload(f"small3d_{n}", c, omega, h, w_out, w, J, srcs, **kw)


def smooth_3d(n: int = 80, nsrc: int = 32, J: int = 16) -> Workload:
    """n^3 smooth random medium c in [1, 2] (Gaussian-filtered white noise, 4-point width,
    min-max mapped, seed 5001), omega = 2 pi 8 at n = 80 (10 points per wavelength at
    c = 1), outer PML 8, interface PML 6, J slabs, `nsrc` sources on one z-plane at
    seeded random (x, y) (seed 5002)."""
    h = 1.0 / n
    s = smoothed_noise((n, n, n), 4.0 * n / 80.0, 5001)
    c = 1.0 + (s - s.min()) / (s.max() - s.min())
    rng = np.random.default_rng(5002)
    z0 = int(rng.integers(n // 4, 3 * n // 4))
    pts = point_sources(n, n, nsrc, 5002 + 1)
    srcs = [(i, l, z0) for (i, l) in pts]
    omega = 2 * math.pi * 8.0 * n / 80.0
    return Workload(f"smooth3d_{n}x{n}x{n}_J{J}", c, omega, h, 8, 6, J, srcs, precision="mixed")


def homogeneous_100() -> Workload:
    """100x100 interior, c = 1, 10 points per wavelength, outer PML 10, J = 4,
    interface PML 8, one point source at the grid centre, complex128."""
    n = 100
    h = 1.0 / n
    return Workload("homogeneous_100x100_J4", np.ones((n, n)), 2 * math.pi * 10.0, h, 10, 8, 4,
                    [(50, 50)], precision="c128")


def lens_1000(nsrc: int = 16) -> Workload:
    """1000x1000 Gaussian lens c = 1 - 0.4 exp(-|r-r0|^2/0.1^2) + smoothed noise of
    standard deviation 0.05; 16 sources on row y = 0.1; J = 32, PML 16 / 12."""
    n = 1000
    h = 1.0 / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    lens = 1.0 - 0.4 * np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.01)
    c = lens + 0.05 * smoothed_noise((n, n), 20.0, 2001)
    srcs = [(int((s + 0.5) * n / nsrc), 100) for s in range(nsrc)]
    return Workload("lens_1000x1000_J32", c, 2 * math.pi * 100.0, h, 16, 12, 32, srcs,
                    precision="mixed")


def layers(n: int = 2000, nsrc: int = 64, seed_medium: int = 3001, seed_src: int = 3002,
         J: Optional[int] = None) -> Workload:
    """n x n grid of random horizontal layers (c uniform in [1.5, 4.0], 10-30 layers),
    omega h = 2 pi / 10 at c = 1.5, `nsrc` uniform-random point sources, J = 64 at
    n = 2000 (scaled with n otherwise), outer PML 16, interface PML 14."""
    h = 1.0 / n
    cy = _layers_1d(n, seed_medium)
    c = np.repeat(cy[:, None], n, axis=1)
    omega = 2 * math.pi * 1.5 / (10 * h)
    if J is None:
        J = max(1, int(round(64 * n / 2000)))
    srcs = point_sources(n, n, nsrc, seed_src)
    return Workload(f"layers_{n}x{n}_J{J}", c, omega, h, 16, 14, J, srcs, precision="mixed")


def layers_uneven_batch() -> List[Workload]:
    """Eight uneven problems: 500^2, 750^2, ..., 2000^2 plus a second 2000^2 with another
    seed, 8 random sources each, J = round(64 n / 2000)."""
    out = []
    sizes = [500, 750, 1000, 1250, 1500, 1750, 2000, 2000]
    for k, n in enumerate(sizes):
        out.append(layers(n=n, nsrc=8, seed_medium=3100 + k, seed_src=3200 + k))
    return out


def smooth_500() -> Workload:
    """500x500 smooth random medium c in [1.5, 3] (Gaussian-smoothed, min-max mapped),
    omega = 2 pi 50, J = 16, 8 sources on the top row, receivers on row 5."""
    n = 500
    h = 1.0 / n
    s = smoothed_noise((n, n), 25.0, 4001)
    c = 1.5 + 1.5 * (s - s.min()) / (s.max() - s.min())
    srcs = [(int((k + 0.5) * n / 8), 0) for k in range(8)]
    wl = Workload("smooth_500x500_J16", c, 2 * math.pi * 50.0, h, 16, 10, 16, srcs,
                  precision="mixed")
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    c_true = c * (1.0 + 0.1 * np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.01))
    rng = np.random.default_rng(4002)
    fd_pts = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(20)]
    wl.extra = {"c_true": c_true, "rec_row": 5, "fd_points": fd_pts}
    return wl


WORKLOADS = {"homogeneous_100": homogeneous_100, "lens_1000": lens_1000, "layers": layers, "smooth_500": smooth_500,
             "smooth_3d": smooth_3d}
