"""3-D parity (7-point stencil, slabs along x) of the HIP path against the CPU oracle on the
same seeded inputs: stencil, slab solves (several Gauss-Jordan panels, a ragged
right-hand-side group), the preconditioner, the reduced operator and both GMRES forms in
both precisions against the direct solution."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.assemble import assemble_global  # noqa: E402
from oracle.dd import StripSolvers, apply_AP_reduced, apply_P  # noqa: E402
from oracle.grid import geometry_from_workload  # noqa: E402
from oracle.solve import solve_dd, solve_dd_reduced, solve_direct  # noqa: E402

DEV = "cuda:0"
TOL_A = 1e-13
TOL_C128 = 1e-10
TOL_C64 = 2e-4
TOL_FIELD = 1e-5


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _rel(a, b):
    """Worst right-hand side of the relative L2 and relative max-norm errors: arrays with
    a leading right-hand-side axis (4-D) are compared one right-hand side at a time, a
    single field (3-D) as one."""
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    if a.ndim == 3:
        a, b = a[None], b[None]
    worst = 0.0
    for k in range(b.shape[0]):
        d = a[k] - b[k]
        worst = max(worst, np.linalg.norm(d) / np.linalg.norm(b[k]), np.abs(d).max() / np.abs(b[k]).max())
    return float(worst)


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.fixture(scope="module")
def case():
    n = 10
    c = 1.0 + 0.3 * np.random.default_rng(17).random((n, n, n))
    wl = W.small3(n=n, J=3, w_out=4, w=3, c=c, nsrc=2, seed=18)
    g = geometry_from_workload(wl)
    return wl, g, assemble_global(g), StripSolvers(g)


def _gpu(wl, prec="c128", mode="full"):
    from paper_1208_3956_amd import Helmholtz
    return Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                     pml_iface_s0=wl.pml_iface_s0,
                     prec=prec, mode=mode, device=DEV).factor()


def test_dims_and_partition(case):
    wl, g, A, S = case
    H = _gpu(wl)
    assert (H.N_x, H.N_y, H.N_z, H.J) == (g.N_x, g.N_y, g.N_z, g.J)
    assert H.beta == list(g.beta) and H.strip_width == [st.W for st in g.strips]
    H.close()


def test_stencil_3d(case):
    wl, g, A, S = case
    H = _gpu(wl)
    rng = np.random.default_rng(1)
    u = _rand(rng, (2,) + g.field_shape)
    f = _rand(rng, (2,) + g.field_shape)
    out = H.apply_A(_t(u), _t(f)).cpu().numpy()
    ref = np.stack([fk - (A @ uk.ravel()).reshape(uk.shape) for uk, fk in zip(u, f)])
    assert _rel(out, ref) < TOL_A
    H.close()


@pytest.mark.parametrize("prec,tol,nrhs", [("c128", TOL_C128, 1), ("c128", TOL_C128, 19),
                                           ("mixed", TOL_C64, 5)])
def test_slab_solve(case, prec, tol, nrhs):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec)
    rng = np.random.default_rng(nrhs)
    for s, st in enumerate(g.strips):
        r = _rand(rng, (nrhs,) + g.strip_shape(st))
        x = H.strip_solve(s, _t(r)).cpu().numpy()
        ref = np.stack([S.solve(s, rk) for rk in r])
        assert _rel(x, ref) < tol, (s, _rel(x, ref))
    H.close()


@pytest.mark.parametrize("prec,tol", [("c128", TOL_C128), ("mixed", TOL_C64)])
def test_apply_P_3d(case, prec, tol):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec)
    rng = np.random.default_rng(4)
    f = _rand(rng, (3,) + g.field_shape)
    pf = H.apply_P(_t(f)).cpu().numpy()
    ref = np.stack([apply_P(g, S, A, fk) for fk in f])
    assert _rel(pf, ref) < tol, _rel(pf, ref)
    H.close()


@pytest.mark.parametrize("prec,tol", [("c128", TOL_C128), ("mixed", TOL_C64)])
def test_apply_AP_reduced_3d(case, prec, tol):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec, mode="reduced")
    rng = np.random.default_rng(6)
    psi = _rand(rng, (2, g.N_z, g.N_y, 2 * (g.J - 1)))
    out = H.apply_AP_reduced(_t(psi)).cpu().numpy()
    ref = np.stack([apply_AP_reduced(g, S, A, pk) for pk in psi])
    assert _rel(out, ref) < tol, _rel(out, ref)
    H.close()


@pytest.mark.parametrize("mode", ["full", "reduced"])
@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_solve_3d_matches_direct(case, mode, prec):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec, mode=mode)
    f = wl.rhs()
    res = H.solve(_t(f), tol=1e-6)
    u = res.u.cpu().numpy()
    ud = solve_direct(g, f, A)
    assert res.status == 0 and max(res.relres) <= 1e-6
    for k in range(f.shape[0]):
        assert _rel(u[k], ud[k]) < TOL_FIELD, (k, _rel(u[k], ud[k]))
    if prec == "c128":
        solver = solve_dd if mode == "full" else solve_dd_reduced
        for k in range(f.shape[0]):
            ref = solver(g, f[k], 1e-6, S=S, A=A)
            assert abs(res.iters[k] - ref.iters) <= 1, (k, res.iters[k], ref.iters)
    H.close()


def test_3d_one_slab_is_one_iteration():
    wl = W.small3(n=8, J=1, w_out=3, w=2, nsrc=1)
    H = _gpu(wl)
    res = H.solve(_t(wl.rhs()), tol=1e-10)
    assert res.iters == [1] and max(res.relres) < 1e-10
    H.close()


def test_factor_path_by_precision(case):
    """complex64 slabs are inverted by the complex64 blocked Gauss-Jordan (its diagonal
    blocks are well conditioned here); complex128 by the FP64 one."""
    wl, g, A, S = case
    H = _gpu(wl, prec="mixed")
    assert H.factor_path == 1
    assert H.factor_slots == wl.J          # a medium that varies with x: one per slab
    H.close()
    H = _gpu(wl, prec="c128")
    assert H.factor_path == 0
    H.close()


@pytest.mark.parametrize("n,J,s", [(40, 16, 7), (40, 16, 15), (20, 4, 1)])
def test_complex64_slab_factor_multiblock(n, J, s):
    """Smooth media: 40^3 (blocks of 840-896 unknowns padded to 896, seven 128-wide column
    blocks) and 20^3 (648 padded to 704: five 128-wide blocks and a last 64-wide one).  Slab
    solves of the complex64 blocked Gauss-Jordan factor against the oracle's SuperLU slab
    solves."""
    from oracle.assemble import assemble_strip
    import scipy.sparse.linalg as spla
    wl = W.smooth_3d(n=n, nsrc=4, J=J)
    g = geometry_from_workload(wl)
    H = _gpu(wl, prec="mixed")
    assert H.factor_path == 1
    st = g.strips[s]
    print(f"slab {s}: {g.strip_shape(st)}", flush=True)
    lu = spla.splu(assemble_strip(g, st).tocsc(), permc_spec="COLAMD")
    rng = np.random.default_rng(40 + s)
    r = _rand(rng, (3,) + g.strip_shape(st))
    x = H.strip_solve(s, _t(r)).cpu().numpy()
    ref = np.stack([lu.solve(rk.ravel()).reshape(rk.shape) for rk in r])
    assert _rel(x, ref) < TOL_C64, _rel(x, ref)
    H.close()


def test_complex64_fp64_route_rounded(case, monkeypatch):
    """The route a complex64 factorisation takes after an ill-conditioned diagonal block
    (FP64 Gauss-Jordan with pivoting over the whole column, rounded to complex64, then
    stored in the 16-row panels of the sweeps), forced from the start: slab solves against
    the oracle's and a solve against the direct solution, at the complex64 bars."""
    wl, g, A, S = case
    monkeypatch.setenv("HELM_FACTOR3_FP64", "1")
    H = _gpu(wl, prec="mixed", mode="reduced")
    assert H.factor_path == 0
    rng = np.random.default_rng(9)
    for s in range(g.J):
        r = _rand(rng, (3,) + g.strip_shape(g.strips[s]))
        x = H.strip_solve(s, _t(r)).cpu().numpy()
        ref = np.stack([S.solve(s, rk) for rk in r])
        assert _rel(x, ref) < TOL_C64, (s, _rel(x, ref))
    f = wl.rhs()
    res = H.solve(_t(f), tol=1e-6)
    ud = solve_direct(g, f, A)
    assert res.status == 0 and max(res.relres) <= 1e-6
    for k in range(f.shape[0]):
        assert _rel(res.u.cpu().numpy()[k], ud[k]) < TOL_FIELD
    H.close()


@pytest.mark.parametrize("n,s", [(60, 7)])
def test_complex64_slab_solve_large(n, s):
    """A sampled slab of the smooth 3-D medium at 60^3 (J = 16: blocks of 17 x 76 = 1292
    unknowns, 98192 per slab), complex64 factor and solve against the oracle's SuperLU
    solve, right-hand side by right-hand side, at the complex64 bar."""
    from oracle.assemble import assemble_strip
    import scipy.sparse.linalg as spla
    wl = W.smooth_3d(n=n, nsrc=2, J=16)
    g = geometry_from_workload(wl)
    H = _gpu(wl, prec="mixed", mode="reduced")
    assert H.factor_path == 1
    st = g.strips[s]
    lu = spla.splu(assemble_strip(g, st).tocsc(), permc_spec="COLAMD")
    rng = np.random.default_rng(60 + s)
    r = _rand(rng, (2,) + g.strip_shape(st))
    x = H.strip_solve(s, _t(r)).cpu().numpy()
    ref = np.stack([lu.solve(rk.ravel()).reshape(rk.shape) for rk in r])
    err = _rel(x, ref)
    print(f"{n}^3 slab {s} {g.strip_shape(st)}: worst relative error {err:.2e}", flush=True)
    assert err < TOL_C64
    H.close()
