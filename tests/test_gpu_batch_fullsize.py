"""The uneven batch at its real sizes: eight layered problems of 500^2 .. 2000^2 (8 sources
each, J = round(64 n / 2000)), complex64-mixed, reduced form, solved concurrently
(helm_solve_batch) as `bench.py --workload layers_uneven_batch` times them: on their own
streams, and with their strip solves fused into multi-problem launches.

Every problem's concurrent solve must equal its solve on its own bit for bit; for one
sampled right-hand side of every problem, the residual f - A u with A assembled by the
oracle must meet 1e-6 and equal the library's own figure; on the 500^2 problem a sampled
right-hand side's field must agree with the oracle's reduced DD-GMRES solution at 1e-10
to the field bar (1e-5)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.assemble import assemble_global  # noqa: E402
from oracle.grid import geometry_from_workload  # noqa: E402
from oracle.solve import solve_dd_reduced  # noqa: E402

DEV = "cuda:0"


def _rel_residual(A, f, u):
    r = f.ravel() - A @ u.ravel()
    return np.linalg.norm(r) / np.linalg.norm(f.ravel())


@pytest.mark.parametrize("fuse", [False, True], ids=["streams", "fused"])
def test_uneven_batch_real_sizes(fuse):
    from paper_1208_3956_amd import Helmholtz, solve_batch
    wls = W.layers_uneven_batch()
    torch.cuda.set_device(0)
    streams = [torch.cuda.Stream(DEV) for _ in wls]
    fs = [torch.from_numpy(wl.rhs()).to(DEV) for wl in wls]
    Hs = [Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                    pml_iface_s0=wl.pml_iface_s0, prec="mixed", mode="reduced", device=DEV,
                    stream=s, batch_fuse=fuse).factor() for wl, s in zip(wls, streams)]
    for H in Hs:
        H.stream.synchronize()
    rb = solve_batch(Hs, fs, 1e-6)
    assert all((r.fused_launches > 0) == fuse for r in rb)
    for k, (H, f, r) in enumerate(zip(Hs, fs, rb)):
        assert r.status == 0 and max(r.relres) <= 1e-6, (k, r.status, max(r.relres))
        r1 = H.solve(f, 1e-6)
        H.stream.synchronize()
        assert r1.iters == r.iters and torch.equal(r1.u, r.u), k
        print(f"problem {k} ({wls[k].n_x}^2, J={wls[k].J}): iterations {sorted(set(r.iters))}",
              flush=True)
    if fuse:
        # bitwise the problems' own solves, which the unfused case checks against the oracle
        for H in Hs:
            H.close()
        return
    rng = np.random.default_rng(77)
    for k, (wl, f, r) in enumerate(zip(wls, fs, rb)):
        g = geometry_from_workload(wl)
        A = assemble_global(g)
        j = int(rng.integers(f.shape[0]))
        fk = f[j].cpu().numpy()
        uk = r.u[j].cpu().numpy()
        rel = _rel_residual(A, fk, uk)
        print(f"problem {k}, rhs {j}: oracle residual {rel:.3e}, library {r.relres[j]:.3e}", flush=True)
        assert rel <= 1e-6
        assert abs(rel - r.relres[j]) <= 1e-9 * max(rel, 1e-30) + 1e-12
        if k == 0:
            ref = solve_dd_reduced(g, fk, 1e-10, A=A)
            d = np.abs(uk - ref.u)
            l2 = np.linalg.norm(uk - ref.u) / np.linalg.norm(ref.u)
            mx = d.max() / np.abs(ref.u).max()
            print(f"500^2 rhs {j}: field vs oracle {l2:.2e} (L2), {mx:.2e} (max)", flush=True)
            assert l2 < 1e-5 and mx < 1e-5
    for H in Hs:
        H.close()
