"""Misfit gradient at the 500^2 smooth-medium workload (J = 16, 8 sources on the top row,
receivers on every point of interior row 5, data from the medium with a +10% Gaussian
blob): helm_grad against the oracle's adjoint gradient with direct solves (the data
also from the oracle), and against central finite differences of the misfit at the 20
seeded points of the workload (step 1e-6 in m = 1/c^2), each misfit evaluated with a
complex128 GPU solve at a 1e-12 residual, compared as one 20-vector."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.grad import gradient, misfit as oracle_misfit  # noqa: E402
from oracle.grid import geometry_from_workload  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def case():
    wl = W.smooth_500()
    print(f"fixture: oracle data and gradient at {wl.name}", flush=True)
    g0 = geometry_from_workload(wl)
    f = wl.rhs()
    n = wl.n_x
    row = wl.extra["rec_row"] + wl.w_out
    rec = np.array([row * wl.N_x + i + wl.w_out for i in range(n)], dtype=np.int64)
    m_true = 1.0 / wl.extra["c_true"] ** 2
    _, U = oracle_misfit(g0, m_true, f, rec, np.zeros((f.shape[0], rec.size), complex))
    d = U[:, rec]
    m = 1.0 / wl.c ** 2
    Jref, gref = gradient(g0, m, f, rec, d)
    return wl, g0, f, rec, d, m, Jref, gref


def _H(wl, g0, c, prec, mode="reduced"):
    from paper_1208_3956_amd import Helmholtz
    return Helmholtz(c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                     pml_iface_s0=wl.pml_iface_s0,
                     pml_cref=g0.c_ref, prec=prec, mode=mode, device=DEV).factor()


@pytest.mark.parametrize("prec,tol,bar", [("c128", 1e-10, 1e-7), ("mixed", 1e-6, 1e-4)])
def test_grad_500_matches_oracle(case, prec, tol, bar):
    wl, g0, f, rec, d, m, Jref, gref = case
    H = _H(wl, g0, wl.c, prec)
    mis, g, its = H.grad(torch.from_numpy(f).to(DEV), torch.from_numpy(rec),
                         torch.from_numpy(d).to(DEV), tol)
    H.close()
    g = g.cpu().numpy()
    err = float(np.linalg.norm(g - gref) / np.linalg.norm(gref))
    print(f"{prec}: misfit {mis:.6e} (oracle {Jref:.6e}), gradient error {err:.2e}, "
          f"iterations {sorted(set(its))}", flush=True)
    assert abs(mis - Jref) / Jref < bar
    assert err < bar


def test_grad_500_matches_finite_differences(case):
    wl, g0, f, rec, d, m, Jref, gref = case
    ft = torch.from_numpy(f).to(DEV)
    rt = torch.from_numpy(rec).to(DEV)
    dt = torch.from_numpy(d).to(DEV)
    H = _H(wl, g0, wl.c, "mixed")
    _, g, _ = H.grad(ft, torch.from_numpy(rec), dt, 1e-8)
    H.close()
    g = g.cpu().numpy()

    def J(mm):
        Hm = _H(wl, g0, 1.0 / np.sqrt(mm), "c128")
        res = Hm.solve(ft, 1e-12)
        Hm.close()
        assert res.status == 0, res.relres
        r = res.u.reshape(f.shape[0], -1)[:, rt] - dt
        return 0.5 * float(torch.sum(torch.abs(r) ** 2))

    eps = 1e-6
    fd, ga = [], []
    for (i, l) in wl.extra["fd_points"]:
        mp = m.copy(); mp[l, i] += eps
        mm = m.copy(); mm[l, i] -= eps
        fd.append((J(mp) - J(mm)) / (2 * eps))
        ga.append(g[l, i])
    fd, ga = np.array(fd), np.array(ga)
    err = float(np.linalg.norm(fd - ga) / np.linalg.norm(ga))
    print(f"finite differences at 20 points: relative error {err:.2e}", flush=True)
    assert err < 1e-4
