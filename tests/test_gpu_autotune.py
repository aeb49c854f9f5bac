"""helm_autotune: the chosen chunk size is one of the candidates, every candidate is
timed, the handle is left factored with it (its strip solves and full solves still meet
the oracle), and the on-disk cache returns the same choice without timing."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.assemble import assemble_global  # noqa: E402
from oracle.grid import geometry_from_workload  # noqa: E402
from oracle.solve import solve_direct  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("prec,mode", [("mixed", "reduced"), ("c128", "full")])
def test_autotune_choice_and_solution(prec, mode, tmp_path):
    from paper_1208_3956_amd import Helmholtz
    c = 1.0 + 0.3 * np.random.default_rng(31).random((60, 60))
    wl = W.small(n=60, J=4, w_out=7, w=5, c=c, nsrc=3, seed=32)
    f = torch.from_numpy(wl.rhs()).to(DEV)
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                  pml_iface_s0=wl.pml_iface_s0,
                  prec=prec, mode=mode, chunk=9, device=DEV)
    cache = str(tmp_path / "tune.json")
    cand = (5, 12, 30, 80)
    out = H.autotune(f, candidates=cand, reps=1, cache=cache)
    assert out["chunk_rows"] in cand and not out["cached"]
    assert sorted(out["ms_per_apply"]) == sorted(cand)
    assert all(t > 0 for t in out["ms_per_apply"].values())
    assert H.chunk_rows == out["chunk_rows"]
    res = H.solve(f, 1e-7)
    assert res.status == 0 and max(res.relres) <= 1e-7
    g = geometry_from_workload(wl)
    ud = solve_direct(g, wl.rhs(), assemble_global(g))
    u = res.u.cpu().numpy()
    for k in range(u.shape[0]):
        assert np.linalg.norm(u[k] - ud[k]) / np.linalg.norm(ud[k]) < 1e-5
    # a second handle of the same shape takes the cached choice without timing
    H2 = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                   pml_iface_s0=wl.pml_iface_s0,
                   prec=prec, mode=mode, chunk=9, device=DEV)
    out2 = H2.autotune(f, candidates=cand, reps=1, cache=cache)
    assert out2["cached"] and out2["chunk_rows"] == out["chunk_rows"]
    res2 = H2.solve(f, 1e-7)
    assert res2.iters == res.iters
    assert torch.equal(res2.u, res.u)
    H.close()
    H2.close()


def test_autotune_3d_is_one_chunk():
    from paper_1208_3956_amd import Helmholtz
    wl = W.small3(n=10, J=2, w_out=4, w=3, nsrc=1)
    f = torch.from_numpy(wl.rhs()).to(DEV)
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                  pml_iface_s0=wl.pml_iface_s0,
                  prec="mixed", mode="reduced", device=DEV)
    out = H.autotune(f, candidates=(8, 16), reps=1, cache=None)
    assert out["chunk_rows"] == H.N_y and H.factored
    res = H.solve(f, 1e-6)
    assert res.status == 0
    H.close()
