"""Misfit and adjoint-state gradient (helm_grad, HelmMisfit) against the oracle's
adjoint gradient with direct solves (itself pinned by central finite differences and the
adjoint identity in test_oracle.py)."""
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
    n = 40
    rng = np.random.default_rng(11)
    c = 1.0 + 0.3 * rng.random((n, n))
    wl = W.small(n=n, J=3, w_out=8, w=6, c=c, nsrc=3, seed=12)
    g0 = geometry_from_workload(wl)
    f = wl.rhs()
    # receivers: interior row 5, one point listed twice, one point inside the outer PML
    rec = [(5 + wl.w_out) * wl.N_x + (i + wl.w_out) for i in range(n)]
    rec += [rec[7], 2 * wl.N_x + 3]
    rec = np.array(rec, dtype=np.int64)
    # data from a perturbed medium (direct solves)
    m_true = 1.0 / (c * (1.0 + 0.05 * rng.random((n, n)))) ** 2
    _, U = oracle_misfit(g0, m_true, f, rec, np.zeros((f.shape[0], rec.size), complex))
    d = U[:, rec]
    m = 1.0 / c ** 2
    Jref, gref = gradient(g0, m, f, rec, d)
    return wl, g0, f, rec, d, m, Jref, gref


def _H(wl, g0, prec, mode, chunk=9):
    from paper_1208_3956_amd import Helmholtz
    return Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                     pml_iface_s0=wl.pml_iface_s0,
                     pml_cref=g0.c_ref, prec=prec, mode=mode, chunk=chunk, device=DEV).factor()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec,mode,tol,bar", [("c128", "full", 1e-11, 1e-8),
                                               ("c128", "reduced", 1e-11, 1e-8),
                                               ("mixed", "reduced", 1e-9, 1e-6)])
def test_grad_matches_oracle(case, prec, mode, tol, bar):
    wl, g0, f, rec, d, m, Jref, gref = case
    H = _H(wl, g0, prec, mode)
    mis, g, its = H.grad(torch.from_numpy(f).to(DEV), torch.from_numpy(rec),
                         torch.from_numpy(d).to(DEV), tol)
    H.close()
    assert abs(mis - Jref) / Jref < bar, (mis, Jref)
    assert _rel(g.cpu().numpy(), gref) < bar, _rel(g.cpu().numpy(), gref)
    assert len(its) == 2 * f.shape[0] and min(its) >= 1


def test_autograd_function(case):
    from paper_1208_3956_amd import misfit
    wl, g0, f, rec, d, m, Jref, gref = case
    mt = torch.from_numpy(m.copy()).to(DEV).requires_grad_(True)
    loss = misfit(mt, torch.from_numpy(f).to(DEV), rec, torch.from_numpy(d).to(DEV),
                  omega=wl.omega, h=wl.h, J=wl.J, pml_outer=wl.w_out, pml_iface=wl.w,
                  pml_power=wl.pml_power, pml_s0=wl.pml_s0, pml_cref=g0.c_ref, tol=1e-11)
    (3.0 * loss).backward()
    assert abs(loss.item() - Jref) / Jref < 1e-8
    assert _rel(mt.grad.cpu().numpy(), 3.0 * gref) < 1e-8


def test_grad_rejects_bad_receiver(case):
    from paper_1208_3956_amd._lib import HelmError, HELM_EINVAL
    wl, g0, f, rec, d, m, Jref, gref = case
    H = _H(wl, g0, "c128", "full")
    bad = rec.copy()
    bad[3] = wl.N_x * wl.N_y
    with pytest.raises(HelmError) as e:
        H.grad(torch.from_numpy(f).to(DEV), torch.from_numpy(bad), torch.from_numpy(d).to(DEV), 1e-8)
    assert e.value.status == HELM_EINVAL
    H.close()
