"""Parity at the benchmark's full size (2000² layered medium, J = 64, 64 right-hand sides,
mixed precision, reduced GMRES, default chunking — the configuration bench.py times), on
outputs the oracle can check one by one:

* the residual f - A u of sampled right-hand sides, with A assembled by the oracle;
* sampled strip solves against the oracle's SuperLU factorisations of the same strips;
* the preconditioner P applied to one right-hand side against the oracle's sweeps.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.assemble import assemble_global, assemble_strip  # noqa: E402
from oracle.dd import StripSolvers, apply_P  # noqa: E402
from oracle.grid import geometry_from_workload  # noqa: E402

DEV = "cuda:0"


def _close(x, ref, tol, what="", rows=None):
    """Every right-hand side within tol in relative L2 and relative max-norm; with rows = m
    also every block of m rows (a y-chunk of the strip solver) within 5 tol."""
    assert x.shape == ref.shape, (what, x.shape, ref.shape)
    for k in range(ref.shape[0]):
        d = x[k] - ref[k]
        l2 = np.linalg.norm(d) / np.linalg.norm(ref[k])
        mx = np.abs(d).max() / np.abs(ref[k]).max()
        assert l2 < tol and mx < tol, (what, k, l2, mx)
        if rows:
            for r0 in range(0, ref.shape[1], rows):
                nb = np.linalg.norm(ref[k][r0:r0 + rows])
                if nb > 0:
                    assert np.linalg.norm(d[r0:r0 + rows]) / nb < 5 * tol, (what, k, r0)


@pytest.fixture(scope="module")
def big():
    wl = W.layers(n=2000, nsrc=64)
    g = geometry_from_workload(wl)
    return wl, g, assemble_global(g)


def _H(wl, prec, mode="reduced"):
    from paper_1208_3956_amd import Helmholtz
    return Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                     pml_iface_s0=wl.pml_iface_s0,
                     prec=prec, mode=mode, device=DEV).factor()


def test_full_size_solve_residual_by_oracle_operator(big):
    wl, g, A = big
    H = _H(wl, "mixed")
    f = wl.rhs()
    res = H.solve(torch.from_numpy(f).to(DEV), tol=1e-6)
    assert res.status == 0 and max(res.relres) <= 1e-6
    for k in (0, 31, 63):
        u = res.u[k].cpu().numpy()
        r = f[k].ravel() - A @ u.ravel()
        rel = np.linalg.norm(r) / np.linalg.norm(f[k])
        assert rel <= 1e-6 * (1 + 1e-9), (k, rel)
        assert abs(rel - res.relres[k]) <= 1e-9 * max(rel, 1e-12) + 1e-15, (k, rel, res.relres[k])
    H.close()


@pytest.mark.parametrize("prec,tol", [("mixed", 2e-4), ("c128", 1e-10)])
def test_full_size_strip_solves(big, prec, tol):
    import scipy.sparse.linalg as spla
    wl, g, A = big
    H = _H(wl, prec)
    k2 = g.k2()
    rng = np.random.default_rng(7)
    for s in (0, 31, 63):
        st = g.strips[s]
        lu = spla.splu(assemble_strip(g, st, k2).tocsc(), permc_spec="COLAMD")
        r = rng.standard_normal((2, g.N_y, st.W)) + 1j * rng.standard_normal((2, g.N_y, st.W))
        x = H.strip_solve(s, torch.from_numpy(r).to(DEV)).cpu().numpy()
        ref = np.stack([lu.solve(rk.ravel()).reshape(rk.shape) for rk in r])
        _close(x, ref, tol, f"strip {s}", rows=H.chunk_rows)
    H.close()


def test_full_size_preconditioner_one_rhs(big):
    wl, g, A = big
    S = StripSolvers(g)
    f = wl.rhs([5])
    ref = apply_P(g, S, A, f[0])
    for prec, tol in (("c128", 1e-10), ("mixed", 2e-4)):
        H = _H(wl, prec, mode="full")
        pf = H.apply_P(torch.from_numpy(f).to(DEV)).cpu().numpy()
        _close(pf, ref[None], tol, f"P {prec}")
        H.close()
