"""The concurrent double sweep P_c (opts.sweep = 1: upward and downward sweeps on f at the
same time, the strips' own sources removed once) against the oracle's form of it, element
by element on the same seeded inputs, right-hand side by right-hand side: P_c itself, its
reduced operator on the columns beta_j - 1, beta_j, and GMRES in both forms and precisions
against the direct solution, with iteration counts against the oracle's."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.assemble import assemble_global  # noqa: E402
from oracle.dd import StripSolvers, apply_AP_concurrent_reduced, apply_P_concurrent  # noqa: E402
from oracle.grid import geometry_from_workload  # noqa: E402
from oracle.solve import solve_dd_concurrent, solve_direct  # noqa: E402

DEV = "cuda:0"


def _close(x, ref, tol, what=""):
    assert x.shape == ref.shape, (what, x.shape, ref.shape)
    for k in range(ref.shape[0]):
        d = x[k] - ref[k]
        l2 = np.linalg.norm(d) / np.linalg.norm(ref[k])
        mx = np.abs(d).max() / np.abs(ref[k]).max()
        assert l2 < tol and mx < tol, (what, k, l2, mx)


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def case():
    c = 1.0 + 0.3 * np.random.default_rng(1).random((44, 44))
    wl = W.small(n=44, J=4, w_out=8, w=6, c=c, nsrc=3, seed=5)
    g = geometry_from_workload(wl)
    return wl, g, assemble_global(g), StripSolvers(g)


def _gpu(wl, prec="c128", mode="reduced", chunk=9, **kw):
    from paper_1208_3956_amd import Helmholtz
    return Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                     pml_iface_s0=wl.pml_iface_s0, prec=prec, mode=mode, chunk=chunk,
                     sweep="concurrent", device=DEV, **kw).factor()


@pytest.mark.parametrize("prec,tol", [("c128", 1e-10), ("mixed", 2e-4)])
def test_concurrent_P(case, prec, tol):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec, mode="full")
    rng = np.random.default_rng(4)
    f = _rand(rng, (5, g.N_y, g.N_x))
    pf = H.apply_P(_t(f)).cpu().numpy()
    ref = np.stack([apply_P_concurrent(g, S, fk) for fk in f])
    _close(pf, ref, tol, "P_c")
    H.close()


@pytest.mark.parametrize("prec,tol", [("c128", 1e-10), ("mixed", 2e-4)])
def test_concurrent_reduced_operator(case, prec, tol):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec)
    rng = np.random.default_rng(6)
    psi = _rand(rng, (3, g.N_y, 2 * (g.J - 1)))
    out = H.apply_AP_reduced(_t(psi)).cpu().numpy()
    ref = np.stack([apply_AP_concurrent_reduced(g, S, A, pk) for pk in psi])
    _close(out, ref, tol, "reduced A P_c")
    H.close()


@pytest.mark.parametrize("mode", ["full", "reduced"])
@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_concurrent_solve(case, mode, prec):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec, mode=mode)
    f = wl.rhs()
    res = H.solve(_t(f), tol=1e-6)
    assert res.status == 0 and max(res.relres) <= 1e-6
    _close(res.u.cpu().numpy(), solve_direct(g, f, A), 1e-5, "field")
    if prec == "c128":
        for k in range(f.shape[0]):
            ref = solve_dd_concurrent(g, f[k], 1e-6, S=S, A=A, mode=mode)
            assert abs(res.iters[k] - ref.iters) <= 1, (k, res.iters[k], ref.iters)
    H.close()


def test_concurrent_graph_replay_equals_eager(case):
    """The reduced operator forks to two more streams and joins them; captured into a HIP
    graph and replayed in every GMRES iteration it must give the kernel-by-kernel result
    bit for bit, replay after replay."""
    wl, g, A, S = case
    f = _t(wl.rhs())
    Hg = _gpu(wl, prec="mixed", graph=True)
    He = _gpu(wl, prec="mixed", graph=False)
    a = [Hg.solve(f, tol=1e-6) for _ in range(3)]
    b = He.solve(f, tol=1e-6)
    for r in a:
        assert r.iters == b.iters and torch.equal(r.u, b.u)
    Hg.close()
    He.close()


def test_concurrent_one_strip_is_one_iteration():
    wl = W.small(n=24, J=1, w_out=6, w=4, nsrc=2)
    H = _gpu(wl, mode="full", chunk=5)
    res = H.solve(_t(wl.rhs()), tol=1e-10)
    assert res.iters == [1] * wl.nrhs and max(res.relres) < 1e-10
    H.close()
