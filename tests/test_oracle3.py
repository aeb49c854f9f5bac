"""Pins for the 3-D oracle (7-point stencil, slabs along x; Sec. 2.2 in three dimensions):
each test checks it against something other than itself (a textbook Kronecker-sum
construction, the closed-form sine-transform solution of the Dirichlet problem, the
invariants of Sec. 2.1-2.3, Theorem 1, brute force)."""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp

import workloads as W
from oracle.assemble import assemble_global, assemble_strip, pml_scaling
from oracle.dd import StripSolvers, apply_AP_reduced, apply_P, reduced_setup, sweep, to_reduced
from oracle.grid import geometry_from_workload, make_geometry
from oracle.solve import solve_dd, solve_dd_reduced, solve_direct


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _geom3(n=10, J=2, w_out=4, w=3, c=None, s0=10.0, ppw=8.0, seed=0):
    h = 1.0 / n
    if c is None:
        c = 1.0 + 0.3 * np.random.default_rng(seed).random((n, n, n))
    om = 2 * math.pi / (ppw * h) * float(np.min(c))
    return make_geometry(c, om, h, w_out, w, J, s0=s0)


def _lap1(N):
    return sp.diags([np.ones(N - 1), -2 * np.ones(N), np.ones(N - 1)], [-1, 0, 1])


def test_7pt_textbook_when_alpha_is_one():
    """No damping (s0 = 0, alpha = 1): -(I(x)I(x)Lx + I(x)Ly(x)I + Lz(x)I(x)I)/h^2 - k^2."""
    g = _geom3(n=6, J=1, w_out=2, s0=0.0)
    A = assemble_global(g).toarray()
    Nz, Ny, Nx = g.field_shape
    I = sp.identity
    L = (sp.kron(I(Nz), sp.kron(I(Ny), _lap1(Nx))) + sp.kron(I(Nz), sp.kron(_lap1(Ny), I(Nx)))
         + sp.kron(_lap1(Nz), sp.kron(I(Ny), I(Nx))))
    ref = (-L / g.h ** 2).toarray() - np.diag(g.k2().ravel())
    assert np.abs(A - ref).max() < 1e-9 * np.abs(ref).max()


def test_7pt_sine_transform_closed_form():
    """alpha = 1, constant k^2: A is diagonalised by the type-I sine transform along each
    axis (eigenvalues (4/h^2) sum sin^2(pi p / (2 (N+1))) - k^2); the oracle's direct solve
    equals that closed form."""
    n, wout = 8, 2
    g = _geom3(n=n, J=1, w_out=wout, s0=0.0, c=np.ones((n, n, n)), ppw=7.3)
    rng = np.random.default_rng(3)
    f = _rand(rng, g.field_shape)
    u = solve_direct(g, f)
    k2 = g.k2()[0, 0, 0]
    lam = 0.0
    for ax, N in enumerate(g.field_shape):
        p = np.arange(1, N + 1)
        s = (4.0 / g.h ** 2) * np.sin(np.pi * p / (2 * (N + 1))) ** 2
        shape = [1, 1, 1]
        shape[ax] = N
        lam = lam + s.reshape(shape)
    lam = lam - k2
    uh = scipy.fft.dstn(f, type=1) / lam
    u_ref = scipy.fft.idstn(uh, type=1)
    assert np.linalg.norm(u - u_ref) < 1e-10 * np.linalg.norm(u_ref)


def test_7pt_pml_operator_is_D_times_symmetric():
    """A = D S with D = alpha_x alpha_y alpha_z and S complex symmetric; a half-point alpha
    taken at the wrong point would break the symmetry."""
    g = _geom3(n=6, J=2, w_out=3, w=2)
    A = assemble_global(g)
    D = pml_scaling(g).ravel()
    S = (sp.diags(1.0 / D) @ A).toarray()
    assert np.abs(S - S.T).max() < 1e-10 * np.abs(S).max()
    st = g.strips[0]
    As = assemble_strip(g, st).toarray()
    assert As.shape[0] == g.N_z * g.N_y * st.W


def test_3d_J1_preconditioner_is_exact_inverse():
    g = _geom3(n=8, J=1, w_out=3)
    A = assemble_global(g)
    S = StripSolvers(g)
    f = _rand(np.random.default_rng(5), g.field_shape)
    pf = apply_P(g, S, A, f)
    assert np.linalg.norm(f - (A @ pf.ravel()).reshape(f.shape)) < 1e-12 * np.linalg.norm(f)


def test_3d_support_of_residuals():
    """f - A v lives on the planes x = beta_j - 1, beta_j; f - A P f and phi on beta_j,
    beta_j + 1 (Sec. 2.1-2.3, the same statements with planes for columns)."""
    g = _geom3(n=12, J=3, w_out=3, w=2)
    A = assemble_global(g)
    S = StripSolvers(g)
    f = _rand(np.random.default_rng(6), g.field_shape)
    v, w, res = sweep(g, S, A, f)
    mg = np.ones(g.N_x, bool); mg[g.residual_columns()] = False
    mr = np.ones(g.N_x, bool); mr[g.reduced_columns()] = False
    sc = np.linalg.norm(f)
    assert np.linalg.norm(res[..., mg]) < 1e-12 * sc
    assert np.linalg.norm(res[..., ~mg]) > 1e-3 * sc
    r = f - (A @ (v + w).ravel()).reshape(f.shape)
    assert np.linalg.norm(r[..., mr]) < 1e-12 * sc
    ut, phi = reduced_setup(g, S, A, f)
    assert np.linalg.norm(phi[..., mr]) < 1e-12 * sc


def _thm1_3d(w):
    n = 16
    rng = np.random.default_rng(8)
    cyz = 1.0 + 0.5 * rng.random((n, n))                       # c(z, y), independent of x
    c = np.repeat(cyz[:, :, None], n, axis=2)
    g = make_geometry(c, 2 * math.pi / (8 / n), 1.0 / n, 5, w, 2)
    A = assemble_global(g)
    S = StripSolvers(g)
    f = np.zeros(g.field_shape, complex)
    f[g.N_z // 2, g.N_y // 2, 7] = f[g.N_z // 3, g.N_y // 3, g.N_x - 8] = n ** 3
    v, ww, _ = sweep(g, S, A, f)
    r = f - (A @ (v + ww).ravel()).reshape(f.shape)
    return np.linalg.norm(r) / np.linalg.norm(f)


def test_3d_theorem1_x_invariant_medium():
    """Theorem 1 (Sec. 3.2) in 3-D: an x-independent medium gives A P = I up to the PML
    reflection, which falls as the interface PML widens."""
    e = [_thm1_3d(w) for w in (2, 4, 6)]
    assert e[0] > e[1] > e[2]
    assert e[2] < 0.05


def test_3d_reduced_form_is_the_same_method():
    g = _geom3(n=10, J=3, w_out=3, w=2)
    A = assemble_global(g)
    S = StripSolvers(g)
    rng = np.random.default_rng(9)
    psi = _rand(rng, (g.N_z, g.N_y, 2 * (g.J - 1)))
    full = np.zeros(g.field_shape, complex)
    full[..., g.reduced_columns()] = psi
    ref = to_reduced(g, (A @ apply_P(g, S, A, full).ravel()).reshape(full.shape))
    # Algorithm 3 starts its sweeps at strip 2 and J-1: for inputs on the reduced planes
    # the result is A P restricted to them
    assert np.linalg.norm(apply_AP_reduced(g, S, A, psi) - ref) < 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("mode", ["full", "reduced"])
def test_3d_dd_gmres_reaches_direct_solution(mode):
    wl = W.small3(n=10, J=2, w_out=4, w=3, nsrc=1,
                  c=1.0 + 0.3 * np.random.default_rng(2).random((10, 10, 10)))
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    f = wl.rhs()[0]
    ud = solve_direct(g, f, A)
    solver = solve_dd if mode == "full" else solve_dd_reduced
    res = solver(g, f, 1e-8, A=A)
    assert res.relres < 1e-8
    assert np.linalg.norm(res.u - ud) < 1e-6 * np.linalg.norm(ud)
    assert res.iters <= 10


def test_3d_workload_shapes():
    wl = W.smooth_3d()
    assert wl.c.shape == (80, 80, 80) and wl.N_x == 96 and wl.nrhs == 32
    assert 1.0 <= wl.c.min() and wl.c.max() <= 2.0
    g = make_geometry(wl.c[:, :, :], wl.omega, wl.h, wl.w_out, wl.w, wl.J)
    # slab widths: 5 core + 1 extra + pads (6 internal, 8 outer at the ends)
    assert [st.W for st in g.strips][:2] == [20, 18] and g.strips[-1].W == 19
