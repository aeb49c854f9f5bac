"""Discrete free-space Green's function of the 5-point Helmholtz lattice (oracle pin).

For the textbook stencil (Sec. 2.2 with alpha = 1) on the infinite lattice,
    (4 u_{m,n} - u_{m+1,n} - u_{m-1,n} - u_{m,n+1} - u_{m,n-1}) / h^2 - k^2 u_{m,n} = delta_{m0} delta_{n0} / h^2,
a Fourier series in n reduces every mode theta to the three-term recurrence
    -u_{m+1} + a u_m - u_{m-1} = delta_{m0},   a(theta) = 4 - 2 cos(theta) - (k h)^2,
whose bounded outgoing solution is u_m = rho^{|m|} / (1/rho - rho) with rho^2 - a rho + 1 = 0
and either |rho| < 1 (evanescent) or rho = e^{i phi}, phi in (0, pi) (outgoing for the
e^{-i omega t} time convention of the paper, cf. its Green formula (i/2k) e^{ik|x-s|}).
Hence
    G(m, n) = (1/pi) int_0^pi cos(n theta) rho(theta)^{|m|} / (1/rho - rho) d theta.
For complex k with Im k > 0 every mode decays and the formula holds with the root of
modulus below one.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad


def _rho(a: complex) -> complex:
    """Root of rho^2 - a rho + 1 = 0 that is outgoing / decaying."""
    a = complex(a)
    d = np.sqrt(a * a / 4.0 - 1.0 + 0j)
    r1, r2 = a / 2 + d, a / 2 - d
    if abs(abs(r1) - 1.0) < 1e-14 and abs(abs(r2) - 1.0) < 1e-14:
        return r1 if r1.imag > 0 else r2
    return r1 if abs(r1) < abs(r2) else r2


def lattice_green(m: int, n: int, kh: complex) -> complex:
    """G(m, n) for source f = 1/h^2 at the origin; kh = k h (real, or complex with
    positive imaginary part)."""
    m, n = abs(int(m)), abs(int(n))
    kh2 = complex(kh) ** 2

    def integrand(theta, part):
        a = 4.0 - 2.0 * math.cos(theta) - kh2
        r = _rho(a)
        val = math.cos(n * theta) * r ** m / (1.0 / r - r)
        return val.real if part == 0 else val.imag

    pts = []
    if abs(kh2.imag) < 1e-15:
        c = 1.0 - kh2.real / 2.0          # a(theta) = 2  <=>  cos(theta) = 1 - (kh)^2/2
        if -1.0 < c < 1.0:
            pts = [math.acos(c)]
    kw = dict(limit=800, epsabs=1e-12, epsrel=1e-10)
    re = quad(integrand, 0.0, math.pi, args=(0,), points=pts or None, **kw)[0]
    im = quad(integrand, 0.0, math.pi, args=(1,), points=pts or None, **kw)[0]
    return complex(re, im) / math.pi
