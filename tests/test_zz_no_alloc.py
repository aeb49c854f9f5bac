"""The allocation-free strip solve (helm_strip_solve_noalloc) against helm_strip_solve,
through the C ABI: two calls in a row, the second with fewer right-hand sides, in both
precisions, 2-D and 3-D, and a call larger than the static 64 MiB workspace rejected with
HELM_EINVAL (the handle still usable)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
WORKSPACE_BYTES = 64 << 20


def _solver(wl, prec):
    from paper_1208_3956_amd import Helmholtz
    return Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                     pml_iface_s0=wl.pml_iface_s0, prec=prec, mode="reduced", chunk=9,
                     device=DEV).factor()


def _noalloc(H, s, r):
    from paper_1208_3956_amd import _lib as L
    x = torch.empty_like(r)
    with torch.cuda.device(H.device):
        st = L.helm_strip_solve_noalloc(H.h, s, r.shape[0], r.data_ptr(), x.data_ptr())
    H.stream.synchronize()
    return st, x


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_noalloc_strip_solve_equals_strip_solve(dim, prec):
    if dim == 2:
        c = 1.0 + 0.3 * np.random.default_rng(1).random((40, 40))
        wl = W.small(n=40, J=3, w_out=8, w=6, c=c, nsrc=2, seed=5)
    else:
        c = 1.0 + 0.3 * np.random.default_rng(17).random((10, 10, 10))
        wl = W.small3(n=10, J=3, w_out=4, w=3, c=c, nsrc=2, seed=18)
    H = _solver(wl, prec)
    rng = np.random.default_rng(3)
    for nrhs in (19, 5):                          # the second call is smaller
        for s in range(H.J):
            shape = (nrhs,) + H.row_shape + (H.strip_width[s],)
            r = torch.from_numpy(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).to(DEV)
            st, x = _noalloc(H, s, r)
            assert st == 0, st
            ref = H.strip_solve(s, r)
            torch.cuda.synchronize()
            # the same kernels on the same input: the same result, bit for bit
            assert torch.equal(x, ref), (nrhs, s, float((x - ref).abs().max()))
    H.close()


def test_noalloc_rejects_more_than_its_workspace():
    from paper_1208_3956_amd._lib import HELM_EINVAL
    c = 1.0 + 0.3 * np.random.default_rng(1).random((40, 40))
    wl = W.small(n=40, J=3, w_out=8, w=6, c=c, nsrc=1, seed=5)
    H = _solver(wl, "c128")
    per_rhs = H.N_y * 64 * 16                    # [row][64] complex128 per right-hand side
    nrhs = WORKSPACE_BYTES // per_rhs + 1
    r = torch.zeros((nrhs, H.N_y, H.strip_width[0]), dtype=torch.complex128, device=DEV)
    st, _ = _noalloc(H, 0, r)
    assert st == HELM_EINVAL
    # the largest call that fits, and the handle afterwards
    rng = np.random.default_rng(4)
    for n in (WORKSPACE_BYTES // per_rhs, 2):
        shape = (n, H.N_y, H.strip_width[0])
        ok = torch.from_numpy(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).to(DEV)
        st, x = _noalloc(H, 0, ok)
        assert st == 0 and torch.equal(x, H.strip_solve(0, ok))
    H.close()
