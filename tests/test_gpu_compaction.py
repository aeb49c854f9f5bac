"""Right-hand sides that have converged leave the GMRES operator's panel: the unconverged
ones are gathered into a panel of the next multiple of 16 and their results moved back.
Within the strip-solver family for panels of more than 4 right-hand sides (the one every
compacted panel uses) each right-hand side is treated alone by every kernel (MFMA columns,
one right-hand side per separator chain, per-right-hand-side reductions), so a batched solve
must give, right-hand side by right-hand side, bitwise the field and the iteration count of
solving it in a panel whose other right-hand sides are zero (they converge at once, and the
panel compacts to 16 before the first iteration).  Panels of at most 4 right-hand sides run
another kernel family (its results agree to rounding, not bitwise).  The panel counters
show the compaction happened."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _pad16(k, nrhs):
    p = (k + 15) // 16 * 16
    return nrhs if (p >= nrhs or k == 0) else p


@pytest.mark.parametrize("mode", ["reduced", "full"])
@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_batched_solve_is_bitwise_the_single_solves(mode, prec):
    from paper_1208_3956_amd import Helmholtz
    c = 1.0 + 0.4 * np.random.default_rng(21).random((48, 48))
    wl = W.small(n=48, J=4, w_out=8, w=6, c=c, nsrc=24, seed=23)
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                  pml_iface_s0=wl.pml_iface_s0, prec=prec, mode=mode, chunk=9,
                  device=DEV).factor()
    f = torch.from_numpy(wl.rhs()).to(DEV)
    nrhs = f.shape[0]
    rb = H.solve(f, 1e-9)
    print(f"{prec}/{mode}: iterations {rb.iters}, restarts {rb.restarts}, panel "
          f"{rb.panel_rhs} of {rb.panel_rhs_full}", flush=True)
    assert rb.status == 0 and max(rb.relres) <= 1e-9
    assert rb.panel_rhs <= rb.panel_rhs_full
    if rb.restarts == 0:
        # one GMRES cycle: iteration k runs the right-hand sides with more than k iterations
        want = sum(_pad16(sum(1 for i in rb.iters if i > k), nrhs) for k in range(max(rb.iters)))
        assert rb.panel_rhs == want, (rb.panel_rhs, want)
    for k in range(nrhs):
        fk = torch.zeros((17,) + tuple(f.shape[1:]), dtype=f.dtype, device=DEV)
        fk[0] = f[k]
        r1 = H.solve(fk, 1e-9)
        assert r1.iters[0] == rb.iters[k], (k, r1.iters[0], rb.iters[k])
        assert torch.equal(r1.u[0], rb.u[k]), k
        assert not bool(r1.u[1:].any())
    H.close()
