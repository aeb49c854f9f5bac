"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by element on
the same seeded inputs.  Sizes span several y-chunks with a ragged last chunk, several
right-hand-side groups with a ragged last group, and the degenerate cases (one strip,
one chunk, two-row chunks)."""
import math

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.assemble import assemble_global  # noqa: E402
from oracle.dd import StripSolvers, apply_AP_reduced, apply_P  # noqa: E402
from oracle.grid import geometry_from_workload  # noqa: E402
from oracle.solve import solve_dd, solve_dd_reduced, solve_direct  # noqa: E402

DEV = "cuda:0"

# floating-point bars: FP64 path ~ round-off times a modest condition number; the
# complex64 path at the preconditioner bar 2e-4 (relative L2)
TOL_A = 1e-13
TOL_STRIP_C128 = 1e-10
TOL_P_C128 = 1e-10
TOL_P_C64 = 2e-4
TOL_FIELD = 1e-5


def _het(n, seed=1, amp=0.3):
    return 1.0 + amp * np.random.default_rng(seed).random((n, n))


def _wl(n=40, J=3, w_out=8, w=6, c=None, nsrc=3, seed=5):
    c = _het(n) if c is None else c
    return W.small(n=n, J=J, w_out=w_out, w=w, c=c, nsrc=nsrc, seed=seed)


def _gpu(wl, prec="c128", mode="full", chunk=9):
    from paper_1208_3956_amd import Helmholtz
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                  pml_iface_s0=wl.pml_iface_s0,
                  prec=prec, mode=mode, chunk=chunk, device=DEV)
    return H.factor()


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _close(x, ref, tol, what="", rows=None):
    """Every right-hand side (leading index) within tol in relative L2 and in relative
    max-norm (max |x - ref| / max |ref|); with rows = m, also every block of m rows (the
    strip solver's y-chunks) within 5 tol in relative L2, so that an error confined to one
    right-hand-side group, chunk or row cannot hide under a norm over everything."""
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
                    eb = np.linalg.norm(d[r0:r0 + rows]) / nb
                    assert eb < 5 * tol, (what, k, r0, eb)


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def case():
    wl = _wl()
    g = geometry_from_workload(wl)
    return wl, g, assemble_global(g), StripSolvers(g)


def test_partition_matches_oracle(case):
    wl, g, A, S = case
    H = _gpu(wl)
    assert H.beta == list(g.beta)
    assert H.strip_width == [st.W for st in g.strips]
    assert H.strip_first == [st.a for st in g.strips]
    H.close()


def test_stencil_apply(case):
    wl, g, A, S = case
    H = _gpu(wl)
    rng = np.random.default_rng(0)
    u = _rand(rng, (3, g.N_y, g.N_x))
    f = _rand(rng, (3, g.N_y, g.N_x))
    out = H.apply_A(_t(u), _t(f)).cpu().numpy()
    ref = np.stack([fk - (A @ uk.ravel()).reshape(uk.shape) for uk, fk in zip(u, f)])
    _close(out, ref, TOL_A, "f - A u")
    out2 = H.apply_A(_t(u)).cpu().numpy()
    _close(out2, f - ref, TOL_A, "A u")
    H.close()


@pytest.mark.parametrize("chunk", [2, 9, 64])
@pytest.mark.parametrize("nrhs", [1, 19])
def test_strip_solve_c128(case, chunk, nrhs):
    wl, g, A, S = case
    H = _gpu(wl, chunk=chunk)
    rng = np.random.default_rng(chunk + nrhs)
    for s, st in enumerate(g.strips):
        r = _rand(rng, (nrhs, g.N_y, st.W))
        x = H.strip_solve(s, _t(r)).cpu().numpy()
        ref = np.stack([S.solve(s, rk) for rk in r])
        _close(x, ref, TOL_STRIP_C128, f"strip {s}", rows=H.chunk_rows)
    H.close()


@pytest.mark.parametrize("chunk", [2, 9, 16, 24])
@pytest.mark.parametrize("nrhs", [5, 19])
def test_strip_solve_mixed(case, chunk, nrhs):
    """complex64 strip solves over chunk sizes (single-row chunks at chunk = 2, a ragged last
    chunk) and ragged right-hand-side groups."""
    wl, g, A, S = case
    H = _gpu(wl, prec="mixed", chunk=chunk)
    rng = np.random.default_rng(3 + chunk + nrhs)
    for s, st in enumerate(g.strips):
        r = _rand(rng, (nrhs, g.N_y, st.W))
        x = H.strip_solve(s, _t(r)).cpu().numpy()
        ref = np.stack([S.solve(s, rk) for rk in r])
        _close(x, ref, TOL_P_C64, f"strip {s}", rows=H.chunk_rows)
    H.close()


@pytest.mark.parametrize("prec,tol", [("c128", TOL_P_C128), ("mixed", TOL_P_C64)])
def test_apply_P(case, prec, tol):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec)
    rng = np.random.default_rng(4)
    f = _rand(rng, (6, g.N_y, g.N_x))
    pf = H.apply_P(_t(f)).cpu().numpy()
    ref = np.stack([apply_P(g, S, A, fk) for fk in f])
    _close(pf, ref, tol, "P")
    H.close()


@pytest.mark.parametrize("prec,tol", [("c128", TOL_P_C128), ("mixed", TOL_P_C64)])
def test_apply_AP_reduced(case, prec, tol):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec, mode="reduced")
    rng = np.random.default_rng(6)
    psi = _rand(rng, (4, g.N_y, 2 * (g.J - 1)))
    out = H.apply_AP_reduced(_t(psi)).cpu().numpy()
    ref = np.stack([apply_AP_reduced(g, S, A, pk) for pk in psi])
    _close(out, ref, tol, "reduced A P")
    H.close()


@pytest.mark.parametrize("prec,tol", [("c128", 1e-9), ("mixed", 1e-3)])
def test_restart_rhs_reduced(case, prec, tol):
    """A restart's reduced right-hand side from both sweeps in the target-only form (the
    support statement of Sec. 2.1) against its definition, (r - A P r) on the reduced
    columns with the oracle's P, for full fields r with nothing zero."""
    from oracle.dd import to_reduced
    wl, g, A, S = case
    H = _gpu(wl, prec=prec, mode="reduced")
    rng = np.random.default_rng(9)
    r = _rand(rng, (3, g.N_y, g.N_x))
    out = H.restart_rhs_reduced(_t(r)).cpu().numpy()
    ref = np.stack([to_reduced(g, rk - (A @ apply_P(g, S, A, rk).ravel()).reshape(rk.shape)) for rk in r])
    err = max(np.linalg.norm(out[k] - ref[k]) / np.linalg.norm(ref[k]) for k in range(len(r)))
    print(f"restart right-hand side ({prec}): relative error {err:.2e}", flush=True)
    _close(out, ref, tol, "restart right-hand side")
    H.close()


def test_restart_rhs_reduced_rejects_one_strip():
    from paper_1208_3956_amd import Helmholtz
    wl = W.small(n=24, J=1, w_out=6, w=4, nsrc=1)
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, prec="c128", mode="reduced",
                  device=DEV).factor()
    with pytest.raises(Exception, match="J = 1"):
        H.restart_rhs_reduced(_t(np.zeros((1, H.N_y, H.N_x), dtype=np.complex128)))
    H.close()


@pytest.mark.parametrize("mode", ["full", "reduced"])
@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_solve_matches_direct(case, mode, prec):
    wl, g, A, S = case
    H = _gpu(wl, prec=prec, mode=mode)
    f = wl.rhs()
    res = H.solve(_t(f), tol=1e-6)
    u = res.u.cpu().numpy()
    ud = solve_direct(g, f, A)
    assert res.status == 0
    assert max(res.relres) <= 1e-6
    _close(u, ud, TOL_FIELD, "field")
    # iteration counts against the oracle's DD-GMRES (MGS vs CGS2 and the mixed
    # precision may move the crossing of the tolerance by one step)
    solver = solve_dd if mode == "full" else solve_dd_reduced
    for k in range(f.shape[0]):
        ref = solver(g, f[k], 1e-6, S=S, A=A)
        assert abs(res.iters[k] - ref.iters) <= 1, (k, res.iters[k], ref.iters)
    H.close()


def test_one_strip_is_one_iteration():
    wl = _wl(n=24, J=1, w_out=6, w=4)
    H = _gpu(wl, chunk=5)
    res = H.solve(_t(wl.rhs()), tol=1e-10)
    assert res.iters == [1] * wl.nrhs and max(res.relres) < 1e-10
    H.close()


def test_homogeneous_100_plain_c128():
    """100x100 homogeneous, J = 4, one source at the centre, complex128."""
    wl = W.homogeneous_100()
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    H = _gpu(wl, chunk=0)
    f = wl.rhs()
    res = H.solve(_t(f), tol=1e-6)
    ud = solve_direct(g, f, A)
    ref = solve_dd(g, f[0], 1e-6, A=A)
    assert res.relres[0] <= 1e-6
    _close(res.u.cpu().numpy(), ud, TOL_FIELD, "field")
    assert abs(res.iters[0] - ref.iters) <= 1
    H.close()


def test_deterministic_and_batch_independent(case):
    wl, g, A, S = case
    H = _gpu(wl, prec="mixed")
    rng = np.random.default_rng(9)
    f = _t(_rand(rng, (5, g.N_y, g.N_x)))
    a = H.apply_P(f).cpu().numpy()
    b = H.apply_P(f).cpu().numpy()
    assert np.array_equal(a, b)
    one = np.concatenate([H.apply_P(f[k:k + 1]).cpu().numpy() for k in range(5)])
    assert _rel(one, a) < 1e-6
    H.close()


def test_solve_before_factor_is_state_error(case):
    from paper_1208_3956_amd import Helmholtz
    from paper_1208_3956_amd._lib import HelmError, HELM_ESTATE
    wl, g, A, S = case
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, device=DEV)
    with pytest.raises(HelmError) as e:
        H.apply_P(_t(np.zeros((1, g.N_y, g.N_x), complex)))
    assert e.value.status == HELM_ESTATE
    H.close()


def test_shape_checks_before_launch(case):
    wl, g, A, S = case
    H = _gpu(wl)
    with pytest.raises(ValueError):
        H.apply_P(torch.zeros((1, g.N_y + 1, g.N_x), dtype=torch.complex128, device=DEV))
    with pytest.raises(TypeError):
        H.apply_P(torch.zeros((1, g.N_y, g.N_x), dtype=torch.complex64, device=DEV))
    H.close()


@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_identical_strips_share_factors(prec):
    """An x-invariant (layered) medium makes every interior strip of one width alike: those
    share one factorisation; every strip's solve and the preconditioner still match the
    oracle, which factors each strip on its own.  A medium that varies with x keeps one
    factorisation per strip."""
    n, J = 60, 6
    cy = 1.0 + 0.5 * np.random.default_rng(3).random(n)
    wl = _wl(n=n, J=J, c=np.repeat(cy[:, None], n, 1))
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    S = StripSolvers(g)
    H = _gpu(wl, prec=prec, chunk=7)
    widths = [st.W for st in g.strips]
    # first and last strips see the outer PML; the interior ones differ only by width
    assert H.factor_slots == 2 + len(set(widths[1:-1])) < J
    slot = H.strip_factor_slot
    assert slot[0] == 0 and all((slot[a] == slot[b]) == (widths[a] == widths[b])
                                for a in range(1, J - 1) for b in range(1, J - 1))
    tol = TOL_STRIP_C128 if prec == "c128" else TOL_P_C64
    rng = np.random.default_rng(12)
    for s, st in enumerate(g.strips):
        r = _rand(rng, (2, g.N_y, st.W))
        x = H.strip_solve(s, _t(r)).cpu().numpy()
        ref = np.stack([S.solve(s, rk) for rk in r])
        _close(x, ref, tol, f"strip {s}", rows=7)
    f = _rand(rng, (2, g.N_y, g.N_x))
    pf = H.apply_P(_t(f)).cpu().numpy()
    ref = np.stack([apply_P(g, S, A, fk) for fk in f])
    _close(pf, ref, TOL_P_C128 if prec == "c128" else TOL_P_C64, "P")
    H.close()
    H = _gpu(_wl(n=n, J=J), prec=prec, chunk=7)
    assert H.factor_slots == J
    H.close()
