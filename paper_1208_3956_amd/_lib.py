"""ctypes binding of libhelm.so (the C ABI in include/helm.h).

Argument marshalling only: every step of the solver runs in the HIP library.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelm.so")

HELM_OK, HELM_EINVAL, HELM_ENOMEM, HELM_EHIP, HELM_ESTATE, HELM_ESINGULAR, HELM_ENOCONV = range(7)
HELM_C128, HELM_MIXED_C64 = 0, 1
HELM_FULL, HELM_REDUCED = 0, 1
STATUS_NAMES = {0: "HELM_OK", 1: "HELM_EINVAL", 2: "HELM_ENOMEM", 3: "HELM_EHIP",
                4: "HELM_ESTATE", 5: "HELM_ESINGULAR", 6: "HELM_ENOCONV"}

# every entry point declared in include/helm.h
EXPORTS = ["helm_default_opts", "helm_setup", "helm_factor", "helm_solve", "helm_apply_P",
           "helm_apply_AP_reduced", "helm_restart_rhs_reduced", "helm_apply_A", "helm_strip_solve", "helm_get_dims",
           "helm_get_partition", "helm_get_chunks", "helm_get_stats", "helm_set_kernel_timing",
           "helm_get_kernel_times", "helm_last_error", "helm_destroy", "helm_grad",
           "helm_solve_batch", "helm_get_dims3", "helm_autotune", "helm_get_factor_path",
           "helm_get_factor_slots", "helm_strip_solve_noalloc", "helm_get_panel_stats",
           "helm_get_fusion_stats"]
KERNEL_CLASSES = ["phase_a", "phase_b", "phase_c", "factor_chunks", "factor_separators",
                  "stencil", "gmres_vectors", "other"]


class HelmOpts(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("pml_outer", ctypes.c_int),
        ("pml_iface", ctypes.c_int),
        ("pml_power", ctypes.c_double),
        ("pml_s0", ctypes.c_double),
        ("pml_cref", ctypes.c_double),
        ("beta", ctypes.POINTER(ctypes.c_int)),
        ("beta_rule", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("mode", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("chunk", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("graph", ctypes.c_int),
        ("pml_iface_s0", ctypes.c_double),
        ("sweep", ctypes.c_int),
        ("transmission", ctypes.c_int),
        ("restart", ctypes.c_int),
        ("batch_fuse", ctypes.c_int),
    ]


class HelmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if libhelm.so is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1208_3956_amd.build` "
                          "(the solver has no non-HIP fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    pint, pdbl = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    L.helm_default_opts.argtypes = [ctypes.POINTER(HelmOpts), ci, ci]
    L.helm_default_opts.restype = None
    L.helm_setup.argtypes = [pdbl, cd, cd, ctypes.POINTER(HelmOpts), ci, ctypes.POINTER(vp)]
    L.helm_factor.argtypes = [vp]
    L.helm_solve.argtypes = [vp, ci, vp, vp, cd, pint, pdbl]
    L.helm_apply_P.argtypes = [vp, ci, vp, vp]
    L.helm_apply_AP_reduced.argtypes = [vp, ci, vp, vp]
    L.helm_restart_rhs_reduced.argtypes = [vp, ci, vp, vp]
    L.helm_apply_A.argtypes = [vp, ci, vp, vp, vp]
    L.helm_solve_batch.argtypes = [ci, ctypes.POINTER(vp), pint, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   cd, pint, pdbl]
    L.helm_grad.argtypes = [vp, ci, vp, ci, vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                            vp, pint]
    L.helm_strip_solve.argtypes = [vp, ci, ci, vp, vp]
    L.helm_strip_solve_noalloc.argtypes = [vp, ci, ci, vp, vp]
    L.helm_autotune.argtypes = [vp, ci, vp, pint, ci, ci, pint, pdbl]
    L.helm_get_factor_path.argtypes = [vp, pint]
    L.helm_get_factor_slots.argtypes = [vp, pint, pint]
    L.helm_get_panel_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    L.helm_get_fusion_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    L.helm_get_dims.argtypes = [vp, pint, pint, pint]
    L.helm_get_dims3.argtypes = [vp, pint, pint, pint, pint]
    L.helm_get_partition.argtypes = [vp, pint, pint, pint]
    L.helm_get_chunks.argtypes = [vp, pint, pint]
    L.helm_get_stats.argtypes = [vp, pint, pint, pdbl]
    L.helm_set_kernel_timing.argtypes = [vp, ci]
    L.helm_get_kernel_times.argtypes = [vp, ci, pint, pdbl]
    L.helm_last_error.argtypes = [vp]
    L.helm_last_error.restype = ctypes.c_char_p
    L.helm_destroy.argtypes = [vp]
    L.helm_destroy.restype = None
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("helm_default_opts", "helm_last_error", "helm_destroy"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def check(status: int, handle=None) -> None:
    if status != HELM_OK:
        msg = lib().helm_last_error(handle)
        raise HelmError(status, msg.decode() if msg else "")


# ---------------------------------------------------------------- same-name wrappers

def helm_default_opts(n_x: int, n_y: int) -> HelmOpts:
    o = HelmOpts()
    lib().helm_default_opts(ctypes.byref(o), int(n_x), int(n_y))
    return o


def helm_setup(c_ptr, omega: float, h: float, opts: HelmOpts, J: int):
    """c_ptr: ctypes pointer to n_y*n_x float64 on the host.  Returns the handle."""
    hdl = ctypes.c_void_p()
    st = lib().helm_setup(c_ptr, float(omega), float(h), ctypes.byref(opts), int(J), ctypes.byref(hdl))
    check(st, None)
    return hdl


def helm_factor(hdl) -> None:
    check(lib().helm_factor(hdl), hdl)


def helm_solve(hdl, nrhs: int, rhs_ptr: int, u_ptr: int, tol: float):
    iters = (ctypes.c_int * nrhs)()
    rel = (ctypes.c_double * nrhs)()
    st = lib().helm_solve(hdl, int(nrhs), ctypes.c_void_p(rhs_ptr), ctypes.c_void_p(u_ptr),
                          float(tol), iters, rel)
    if st not in (HELM_OK, HELM_ENOCONV):
        check(st, hdl)
    return st, list(iters), list(rel)


def helm_autotune(hdl, nrhs: int, rhs_ptr: int, cand, reps: int):
    """Returns (chosen rows per chunk, milliseconds per application for each candidate)."""
    n = len(cand)
    C = (ctypes.c_int * n)(*[int(c) for c in cand])
    ms = (ctypes.c_double * n)()
    best = ctypes.c_int(0)
    check(lib().helm_autotune(hdl, int(nrhs), ctypes.c_void_p(rhs_ptr), C, n, int(reps),
                              ctypes.byref(best), ms), hdl)
    return best.value, list(ms)


def helm_apply_P(hdl, nrhs: int, f_ptr: int, out_ptr: int) -> None:
    check(lib().helm_apply_P(hdl, int(nrhs), ctypes.c_void_p(f_ptr), ctypes.c_void_p(out_ptr)), hdl)


def helm_apply_AP_reduced(hdl, nrhs: int, psi_ptr: int, out_ptr: int) -> None:
    check(lib().helm_apply_AP_reduced(hdl, int(nrhs), ctypes.c_void_p(psi_ptr),
                                      ctypes.c_void_p(out_ptr)), hdl)


def helm_restart_rhs_reduced(hdl, nrhs: int, r_ptr: int, b_ptr: int) -> None:
    check(lib().helm_restart_rhs_reduced(hdl, int(nrhs), ctypes.c_void_p(r_ptr),
                                         ctypes.c_void_p(b_ptr)), hdl)


def helm_solve_batch(hdls, nrhs, rhs_ptrs, u_ptrs, tol: float):
    """Returns (status, iterations, relres) over all right-hand sides, problem by problem."""
    n = len(hdls)
    tot = int(sum(nrhs))
    H = (ctypes.c_void_p * n)(*hdls)
    NR = (ctypes.c_int * n)(*[int(k) for k in nrhs])
    R = (ctypes.c_void_p * n)(*rhs_ptrs)
    U = (ctypes.c_void_p * n)(*u_ptrs)
    its = (ctypes.c_int * tot)()
    rel = (ctypes.c_double * tot)()
    st = lib().helm_solve_batch(n, H, NR, R, U, float(tol), its, rel)
    if st not in (HELM_OK, HELM_ENOCONV):
        bad = next((h for h in hdls if helm_last_error(h)), hdls[0])
        check(st, bad)
    return st, list(its), list(rel)


def helm_grad(hdl, nsrc: int, src_ptr: int, nrec: int, rec_ptr: int, d_ptr: int, tol: float,
              grad_ptr: int):
    """Returns (status, misfit, iterations [forward..., adjoint...])."""
    mis = ctypes.c_double(0.0)
    its = (ctypes.c_int * (2 * nsrc))()
    st = lib().helm_grad(hdl, int(nsrc), ctypes.c_void_p(src_ptr), int(nrec), ctypes.c_void_p(rec_ptr),
                         ctypes.c_void_p(d_ptr), float(tol), ctypes.byref(mis), ctypes.c_void_p(grad_ptr),
                         its)
    if st not in (HELM_OK, HELM_ENOCONV):
        check(st, hdl)
    return st, mis.value, list(its)


def helm_apply_A(hdl, nrhs: int, u_ptr: int, f_ptr, out_ptr: int) -> None:
    check(lib().helm_apply_A(hdl, int(nrhs), ctypes.c_void_p(u_ptr),
                             ctypes.c_void_p(f_ptr) if f_ptr else None, ctypes.c_void_p(out_ptr)), hdl)


def helm_strip_solve(hdl, strip: int, nrhs: int, r_ptr: int, x_ptr: int) -> None:
    check(lib().helm_strip_solve(hdl, int(strip), int(nrhs), ctypes.c_void_p(r_ptr),
                                 ctypes.c_void_p(x_ptr)), hdl)


def helm_strip_solve_noalloc(hdl, strip: int, nrhs: int, r_ptr: int, x_ptr: int) -> int:
    """Returns the status (HELM_EINVAL for a call larger than the static workspace)."""
    return lib().helm_strip_solve_noalloc(hdl, int(strip), int(nrhs), ctypes.c_void_p(r_ptr),
                                          ctypes.c_void_p(x_ptr))


def helm_get_dims(hdl):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib().helm_get_dims(hdl, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), hdl)
    return a.value, b.value, c.value


def helm_get_partition(hdl, J: int):
    beta = (ctypes.c_int * (J + 1))()
    first = (ctypes.c_int * J)()
    width = (ctypes.c_int * J)()
    check(lib().helm_get_partition(hdl, beta, first, width), hdl)
    return list(beta), list(first), list(width)


def helm_get_chunks(hdl):
    m, p = ctypes.c_int(), ctypes.c_int()
    check(lib().helm_get_chunks(hdl, ctypes.byref(m), ctypes.byref(p)), hdl)
    return m.value, p.value


def helm_get_factor_path(hdl) -> int:
    p = ctypes.c_int()
    check(lib().helm_get_factor_path(hdl, ctypes.byref(p)), hdl)
    return p.value


def helm_get_factor_slots(hdl, J: int):
    """Returns (number of stored factorisations, the slot of each strip)."""
    p = ctypes.c_int()
    sl = (ctypes.c_int * J)()
    check(lib().helm_get_factor_slots(hdl, ctypes.byref(p), sl), hdl)
    return p.value, list(sl)


def helm_get_stats(hdl):
    a, r, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    check(lib().helm_get_stats(hdl, ctypes.byref(a), ctypes.byref(r), ctypes.byref(ms)), hdl)
    return a.value, r.value, ms.value


def helm_get_panel_stats(hdl):
    """(right-hand sides through the GMRES operator, the same without panel compaction)."""
    a, b = ctypes.c_longlong(), ctypes.c_longlong()
    check(lib().helm_get_panel_stats(hdl, ctypes.byref(a), ctypes.byref(b)), hdl)
    return a.value, b.value


def helm_get_fusion_stats(hdl):
    """(multi-problem strip-solve launches, strip solves launched alone) of the last batch."""
    a, b = ctypes.c_longlong(), ctypes.c_longlong()
    check(lib().helm_get_fusion_stats(hdl, ctypes.byref(a), ctypes.byref(b)), hdl)
    return a.value, b.value


def helm_set_kernel_timing(hdl, mask: int) -> None:
    """mask: bit c times kernel class KERNEL_CLASSES[c]; 0 disables timing."""
    check(lib().helm_set_kernel_timing(hdl, int(mask) & 0xFF), hdl)


def helm_get_kernel_times(hdl) -> dict:
    n = len(KERNEL_CLASSES)
    cnt = (ctypes.c_int * n)()
    ms = (ctypes.c_double * n)()
    check(lib().helm_get_kernel_times(hdl, n, cnt, ms), hdl)
    return {k: (cnt[i], ms[i]) for i, k in enumerate(KERNEL_CLASSES)}


def helm_get_dims3(hdl):
    nx, ny, nz, J = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib().helm_get_dims3(hdl, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(nz), ctypes.byref(J)), hdl)
    return nx.value, ny.value, nz.value, J.value


def helm_last_error(hdl) -> str:
    m = lib().helm_last_error(hdl)
    return m.decode() if m else ""


def helm_destroy(hdl) -> None:
    lib().helm_destroy(hdl)
