"""GPU regression and robustness tests through the C ABI: workspace reuse across
right-hand-side counts, restarts with Krylov recycling, the iteration cap, and the
paper's own partition rule (eq. define_beta_j).  Fields are compared with the oracle's
direct solution and preconditioner, right-hand side by right-hand side."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.assemble import assemble_global  # noqa: E402
from oracle.dd import StripSolvers, apply_P  # noqa: E402
from oracle.grid import geometry_from_workload, partition  # noqa: E402
from oracle.solve import solve_direct  # noqa: E402

DEV = "cuda:0"


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _per_rhs(x, ref, tol, what):
    """Relative L2 and relative max-norm error of every right-hand side below tol."""
    for k in range(ref.shape[0]):
        d = x[k] - ref[k]
        l2 = np.linalg.norm(d) / np.linalg.norm(ref[k])
        mx = np.abs(d).max() / np.abs(ref[k]).max()
        assert l2 < tol and mx < tol, (what, k, l2, mx)


def _wl(n=40, J=3, w_out=8, w=6, nsrc=6, seed=5, s0i=None):
    c = 1.0 + 0.3 * np.random.default_rng(1).random((n, n))
    wl = W.small(n=n, J=J, w_out=w_out, w=w, c=c, nsrc=nsrc, seed=seed)
    wl.pml_iface_s0 = s0i
    return wl


def _gpu(wl, prec="mixed", mode="reduced", chunk=9, **kw):
    from paper_1208_3956_amd import Helmholtz
    return Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                     pml_iface_s0=wl.pml_iface_s0, prec=prec, mode=mode, chunk=chunk,
                     device=DEV, **kw).factor()


def test_gmres_buffers_follow_the_rhs_count():
    """autotune(k) sizes the sweep buffers for k right-hand sides; a following solve of one
    right-hand side must not leave the GMRES buffers at one when a solve of k comes next."""
    wl = _wl()
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    f = wl.rhs()
    ud = solve_direct(g, f, A)
    H = _gpu(wl)
    H.autotune(_t(f), candidates=(7, 9), reps=1, cache=None)
    r1 = H.solve(_t(f[:1]), tol=1e-6)
    assert r1.status == 0 and r1.relres[0] <= 1e-6
    rk = H.solve(_t(f), tol=1e-6)
    assert rk.status == 0 and max(rk.relres) <= 1e-6
    _per_rhs(rk.u.cpu().numpy(), ud, 1e-5, "solve(k) after solve(1)")
    H.close()


def test_recycling_restart_then_more_rhs():
    """Weak interface pads give a first GMRES cycle of about 20 steps; complex64 at tol
    1e-9 forces restarts, so the restart recycles the first cycle's Krylov space.  A solve
    of one right-hand side with recycling, then one of four, must both converge (the
    recycled basis is kept at the capacity of the GMRES basis)."""
    wl = _wl(n=48, J=4, w=4, nsrc=4, s0i=0.5)
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    f = wl.rhs()
    ud = solve_direct(g, f, A)
    H = _gpu(wl, chunk=7)
    r1 = H.solve(_t(f[:1]), tol=1e-9)
    print(f"one rhs: iterations {r1.iters}, restarts {r1.restarts}, relres {r1.relres}", flush=True)
    assert r1.status == 0 and r1.relres[0] <= 1e-9
    assert r1.iters[0] >= 16 and r1.restarts >= 1          # the recycling path was taken
    _per_rhs(r1.u.cpu().numpy(), ud[:1], 1e-7, "recycled solve, 1 rhs")
    r4 = H.solve(_t(f), tol=1e-9)
    print(f"four rhs: iterations {r4.iters}, restarts {r4.restarts}", flush=True)
    assert r4.status == 0 and max(r4.relres) <= 1e-9
    _per_rhs(r4.u.cpu().numpy(), ud, 1e-7, "recycled solve, 4 rhs")
    H.close()


def test_augmented_cycle_then_plain_restart():
    """tol 1e-12 in complex64 needs at least two restarts: the first recycles, the second
    starts plainly (an augmented cycle's Hessenberg matrix is that of the projected
    operator).  The solve must reach the tolerance without running away in restarts."""
    wl = _wl(n=48, J=4, w=4, nsrc=2, s0i=0.5)
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    f = wl.rhs()
    ud = solve_direct(g, f, A)
    H = _gpu(wl, chunk=7)
    r = H.solve(_t(f), tol=1e-12)
    print(f"iterations {r.iters}, restarts {r.restarts}, relres {r.relres}", flush=True)
    assert r.status == 0 and max(r.relres) <= 1e-12
    assert 2 <= r.restarts <= 5
    _per_rhs(r.u.cpu().numpy(), ud, 1e-9, "two restarts")
    H.close()


@pytest.mark.parametrize("mode", ["full", "reduced"])
def test_iteration_cap_reports_enoconv(mode):
    """max_iter = 1 cannot reach 1e-10: HELM_ENOCONV, with the explicit residual of the
    best iterate reported (finite, below the starting residual)."""
    from paper_1208_3956_amd._lib import HELM_ENOCONV
    wl = _wl(nsrc=2)
    H = _gpu(wl, prec="c128", mode=mode, max_iter=1)
    r = H.solve(_t(wl.rhs()), tol=1e-10)
    assert r.status == HELM_ENOCONV
    assert all(np.isfinite(x) and 1e-10 < x < 1.0 for x in r.relres), r.relres
    u = r.u.cpu().numpy()
    assert np.all(np.isfinite(u))
    H.close()


@pytest.mark.parametrize("prec,tol", [("c128", 1e-10), ("mixed", 2e-4)])
def test_paper_partition_rule(prec, tol):
    """beta_rule = 1 places the interfaces by eq. define_beta_j; the library's partition
    equals the oracle's, and P and the solve match the oracle on it."""
    wl = _wl(n=56, J=4, w=5, nsrc=3)
    gp = geometry_from_workload(wl)
    b = partition(wl.n_x, wl.w_out, wl.J, wl.w, rule="paper")
    assert list(b) != list(gp.beta)          # the two rules differ on this grid
    wl.beta = [int(x) for x in b[1:-1]]
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    S = StripSolvers(g)
    H = _gpu(wl, prec=prec, mode="reduced", beta_rule=1)
    assert H.beta == list(b)
    assert H.strip_width == [st.W for st in g.strips]
    f = wl.rhs()
    rng = np.random.default_rng(2)
    x = f + 0.1 * (rng.standard_normal(f.shape) + 1j * rng.standard_normal(f.shape)) / wl.h ** 2
    pf = H.apply_P(_t(x)).cpu().numpy()
    ref = np.stack([apply_P(g, S, A, xk) for xk in x])
    _per_rhs(pf, ref, tol, "P, paper partition")
    res = H.solve(_t(f), tol=1e-6)
    assert res.status == 0 and max(res.relres) <= 1e-6
    _per_rhs(res.u.cpu().numpy(), solve_direct(g, f, A), 1e-5, "solve, paper partition")
    H.close()


def test_resonant_strip_reports_esingular():
    """Without PML (s0 = 0) a strip is a real Dirichlet problem; with k^2 at an eigenvalue of
    its first y-block T = T_x + (2/h^2 - k^2) I (T_x the 1-D second difference over the W
    columns, eigenvalues 4 sin^2(m pi / (2 (W + 1))) / h^2) that block is singular.  The
    factorisation must report HELM_ESINGULAR instead of solving with a meaningless inverse;
    k moved off the eigenvalue by 1% factors normally."""
    import math
    from paper_1208_3956_amd import Helmholtz
    from paper_1208_3956_amd._lib import HelmError, HELM_ESINGULAR
    n, w_out = 10, 1
    h = 1.0 / n
    W_ = n + 2 * w_out                                   # J = 1: the strip is the padded grid
    k2 = 2.0 / h ** 2 + 4.0 * math.sin(math.pi / (2 * (W_ + 1))) ** 2 / h ** 2
    for scale, singular in ((1.0, True), (1.01, False)):
        H = Helmholtz(np.ones((n, n)), math.sqrt(k2 * scale), h, 1, pml_outer=w_out, pml_iface=1,
                      pml_s0=0.0, prec="c128", mode="full", device=DEV)
        if singular:
            with pytest.raises(HelmError) as e:
                H.factor()
            assert e.value.status == HELM_ESINGULAR, e.value
            print(f"resonant strip: {e.value}", flush=True)
        else:
            H.factor()
        H.close()
