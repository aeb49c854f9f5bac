"""Graph replay of the reduced operator and concurrent solves of uneven problems.

Graph: a solve replays the captured Algorithm 3 once per GMRES iteration (with the
program's own eager work and host synchronisations between replays); its iterations and
field must equal the kernel-by-kernel solve bit for bit, on two consecutive solves and
after a change of the right-hand-side count (a new capture).
Batch: problems of different sizes solved concurrently on their own streams must equal
their individual solves bit for bit and the oracle's direct solution to the field bar."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.assemble import assemble_global  # noqa: E402
from oracle.grid import geometry_from_workload  # noqa: E402
from oracle.solve import solve_direct  # noqa: E402

DEV = "cuda:0"


def _wl(n, J, seed):
    c = 1.0 + 0.3 * np.random.default_rng(seed).random((n, n))
    return W.small(n=n, J=J, w_out=7, w=5, c=c, nsrc=3, seed=seed + 1)


def _H(wl, prec, graph, stream=None, chunk=9):
    from paper_1208_3956_amd import Helmholtz
    return Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                     pml_iface_s0=wl.pml_iface_s0,
                     prec=prec, mode="reduced", chunk=chunk, device=DEV, stream=stream,
                     graph=graph).factor()


@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_graph_replay_equals_eager(prec):
    wl = _wl(48, 4, 21)
    f = torch.from_numpy(wl.rhs()).to(DEV)
    He = _H(wl, prec, graph=False)
    Hg = _H(wl, prec, graph=True)
    # both handles see the same sequence of solves (the complex64 path adapts its first
    # GMRES cycle to what earlier solves measured)
    for rep in range(2):
        ref = He.solve(f, 1e-8)
        got = Hg.solve(f, 1e-8)
        assert got.iters == ref.iters, (rep, got.iters, ref.iters)
        assert torch.equal(got.u, ref.u), rep
    # a different right-hand-side count forces a new capture
    ref1 = He.solve(f[1:2], 1e-8)
    got1 = Hg.solve(f[1:2], 1e-8)
    assert got1.iters == ref1.iters and torch.equal(got1.u, ref1.u)
    ref = He.solve(f, 1e-8)
    got = Hg.solve(f, 1e-8)
    assert got.iters == ref.iters and torch.equal(got.u, ref.u)
    He.close()
    Hg.close()


def test_graph_after_refactor():
    """Re-factoring frees and reallocates the factors; the next solve must capture the
    operator again instead of replaying launches that point at the old factors."""
    wl = _wl(40, 3, 25)
    f = torch.from_numpy(wl.rhs()).to(DEV)
    He = _H(wl, "mixed", graph=False)
    Hg = _H(wl, "mixed", graph=True)
    for rep in range(3):
        ref = He.solve(f, 1e-8)
        got = Hg.solve(f, 1e-8)
        assert got.iters == ref.iters and torch.equal(got.u, ref.u), rep
        Hg.factor()
        He.factor()
    He.close()
    Hg.close()


def test_solve_batch_uneven_problems():
    from paper_1208_3956_amd import solve_batch
    wls = [_wl(40, 3, 31), _wl(64, 5, 33), _wl(32, 2, 35)]
    streams = [torch.cuda.Stream(DEV) for _ in wls]
    Hs = [_H(wl, "mixed", True, stream=s) for wl, s in zip(wls, streams)]
    Hone = [_H(wl, "mixed", True) for wl in wls]          # same history, solved one by one
    fs = [torch.from_numpy(wl.rhs()).to(DEV) for wl in wls]
    res = solve_batch(Hs, fs, 1e-6)
    for wl, H1, f, r in zip(wls, Hone, fs, res):
        one = H1.solve(f, 1e-6)
        assert r.iters == one.iters and torch.equal(r.u, one.u)
        assert max(r.relres) <= 1e-6
        g = geometry_from_workload(wl)
        ud = solve_direct(g, wl.rhs(), assemble_global(g))
        err = max(np.linalg.norm(r.u.cpu().numpy()[k] - ud[k]) / np.linalg.norm(ud[k])
                  for k in range(ud.shape[0]))
        assert err < 1e-5, err
    for H in Hs + Hone:
        H.close()


def _fused_case(mode, precs, seeds=(51, 53, 55), sizes=((40, 3), (64, 5), (48, 4))):
    """Problems of different sizes with 6 right-hand sides each (panels of more than 4 take
    the fused launches), each problem also solved on its own by a second handle."""
    from paper_1208_3956_amd import Helmholtz
    wls, Hs, Hone = [], [], []
    for (n, J), seed, prec in zip(sizes, seeds, precs):
        c = 1.0 + 0.3 * np.random.default_rng(seed).random((n, n))
        wl = W.small(n=n, J=J, w_out=7, w=5, c=c, nsrc=6, seed=seed + 1)
        mk = lambda st: Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power,
                                  wl.pml_s0, pml_iface_s0=wl.pml_iface_s0, prec=prec, mode=mode,
                                  chunk=9, device=DEV, stream=st, batch_fuse=True).factor()
        wls.append(wl)
        Hs.append(mk(torch.cuda.Stream(DEV)))
        Hone.append(mk(None))
    return wls, Hs, Hone


@pytest.mark.parametrize("mode", ["reduced", "full"])
def test_solve_batch_fuses_strip_solves(mode):
    """Three complex64 problems of different sizes and strip counts: their strip solves run
    as multi-problem launches (one per phase and sweep step), and every problem's field and
    iteration counts equal its own helm_solve bit for bit."""
    from paper_1208_3956_amd import solve_batch
    wls, Hs, Hone = _fused_case(mode, ["mixed"] * 3)
    fs = [torch.from_numpy(wl.rhs()).to(DEV) for wl in wls]
    res = solve_batch(Hs, fs, 1e-6)
    print(f"{mode}: fused launches {[r.fused_launches for r in res]}, alone "
          f"{[r.unfused_launches for r in res]}, iterations {[r.iters for r in res]}", flush=True)
    for wl, H1, f, r in zip(wls, Hone, fs, res):
        assert r.fused_launches > 0
        one = H1.solve(f, 1e-6)
        assert r.iters == one.iters and torch.equal(r.u, one.u)
        assert max(r.relres) <= 1e-6
        g = geometry_from_workload(wl)
        ud = solve_direct(g, wl.rhs(), assemble_global(g))
        err = max(np.linalg.norm(r.u.cpu().numpy()[k] - ud[k]) / np.linalg.norm(ud[k])
                  for k in range(ud.shape[0]))
        assert err < 1e-5, err
    for H in Hs + Hone:
        H.close()


def test_solve_batch_fuses_only_eligible_problems():
    """A complex128 problem in the batch runs on its own stream and thread; the two
    complex64 problems fuse; all three equal their own solves bit for bit."""
    from paper_1208_3956_amd import solve_batch
    wls, Hs, Hone = _fused_case("reduced", ["mixed", "c128", "mixed"])
    fs = [torch.from_numpy(wl.rhs()).to(DEV) for wl in wls]
    res = solve_batch(Hs, fs, 1e-6)
    assert res[0].fused_launches > 0 and res[2].fused_launches > 0
    assert res[1].fused_launches == 0 and res[1].unfused_launches == 0
    for H1, f, r in zip(Hone, fs, res):
        one = H1.solve(f, 1e-6)
        assert r.iters == one.iters and torch.equal(r.u, one.u)
    for H in Hs + Hone:
        H.close()


def test_solve_batch_rejects_repeated_handle():
    from paper_1208_3956_amd import solve_batch
    from paper_1208_3956_amd._lib import HelmError
    wl = _wl(32, 2, 41)
    H = _H(wl, "c128", True)
    f = torch.from_numpy(wl.rhs()).to(DEV)
    with pytest.raises(HelmError):
        solve_batch([H, H], [f, f], 1e-6)
    H.close()


def test_kernel_timing_class_mask():
    """Timing only some kernel classes: every launch is still counted, only the masked
    classes accumulate time, and the field is the untimed one bit for bit."""
    wl = _wl(48, 4, 31)
    f = torch.from_numpy(wl.rhs()).to(DEV)
    H = _H(wl, "mixed", graph=False)
    ref = H.solve(f, 1e-6)
    H2 = _H(wl, "mixed", graph=False)
    H2.set_kernel_timing(True, classes=["phase_a"])
    res = H2.solve(f, 1e-6)
    kt = H2.kernel_times()
    H2.set_kernel_timing(False)
    assert res.iters == ref.iters and torch.equal(res.u, ref.u)
    assert kt["phase_a"][0] > 0 and kt["phase_a"][1] > 0
    assert kt["stencil"][0] > 0 and kt["stencil"][1] == 0
    assert kt["phase_c"][0] > 0 and kt["phase_c"][1] == 0
    H.close()
    H2.close()
