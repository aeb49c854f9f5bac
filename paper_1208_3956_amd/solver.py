"""Torch-facing wrapper of the HIP Helmholtz library.

PyTorch supplies device memory and the HIP stream; every computation runs in
libhelm.so.  Shapes and dtypes are checked here before anything is launched.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


@dataclass
class SolveResult:
    u: torch.Tensor
    iters: list
    relres: list
    status: int
    ap_applies: int
    restarts: int
    ms: float
    # right-hand sides through the GMRES operator (converged ones leave its panel), and the
    # same count had they stayed
    panel_rhs: int = 0
    panel_rhs_full: int = 0
    # solve_batch: multi-problem strip-solve launches and strip solves launched alone
    fused_launches: int = 0
    unfused_launches: int = 0


class Helmholtz:
    """One discretised 2-D or 3-D Helmholtz problem with its strip (slab) factors.

    c          interior wave speed, (n_y, n_x) or (n_z, n_y, n_x) float64 (numpy or torch;
               copied to the host); 3-D uses the 7-point stencil and slabs along x
    omega, h   angular frequency and grid spacing
    J          number of strips along x
    pml_outer  outer PML width (cells); pml_iface: interface PML width w
    pml_s0     strength of the outer PML (part of A: changes the solution)
    pml_iface_s0  strength of the interface pads (part of P only: changes iterations);
               None = 2.5 x pml_iface (the same damping per cell for every width)
    beta_rule  partition when beta is None: 0 = even split of the interior,
               1 = the paper's rule (eq. define_beta_j)
    sweep      "double" (the paper's P) or "concurrent" (P_c: upward and downward sweeps
               on f at the same time on separate streams)
    transmission  "pml" (the paper's method) or "robin" (the comparison method of Sec. 4.4:
               unpadded subdomains with first-order absorbing conditions; 2-D, full form;
               with sweep="concurrent" the concurrent sweeps of Sec. 3.1, step n solving
               subdomains n and J + 1 - n with two-sided Robin data)
    restart    GMRES cycle length (0 = library default: 60 reduced, 30 full)
    batch_fuse in solve_batch, fuse this problem's strip solves with the other problems
               that set it (lockstep multi-problem launches) instead of its own stream
    prec       "c128" or "mixed" (complex64 strip factors and sweeps, FP64 GMRES)
    mode       "full" or "reduced" (GMRES on the interface columns, Algorithms 2-5)
    chunk      rows per chunk of the y-partitioned strip solver (0 = library default)
    stream     torch.cuda.Stream for all of the handle's work (default: the current stream)
    graph      replay the reduced-form operator from a captured HIP graph (reduced mode)
    """

    def __init__(self, c, omega: float, h: float, J: int, pml_outer: int = 16,
                 pml_iface: int = 8, pml_power: float = 2.0, pml_s0: float = 10.0,
                 pml_cref: float = 0.0, prec: str = "c128", mode: str = "full",
                 max_iter: int = 200, chunk: int = 0, beta: Optional[Sequence[int]] = None,
                 device="cuda:0", stream=None, graph: bool = True,
                 pml_iface_s0: Optional[float] = None,
                 beta_rule: int = 0, sweep: str = "double", transmission: str = "pml",
                 restart: int = 0, batch_fuse: bool = False):
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on a HIP device (cuda:N in torch)")
        c = c.detach().cpu().numpy() if isinstance(c, torch.Tensor) else np.asarray(c)
        self._c = np.ascontiguousarray(c, dtype=np.float64)
        if self._c.ndim not in (2, 3):
            raise ValueError("c must be a (n_y, n_x) or (n_z, n_y, n_x) array")
        n_y, n_x = self._c.shape[-2:]
        o = L.helm_default_opts(n_x, n_y)
        if self._c.ndim == 3:
            o.dim = 3
            o.n[2] = int(self._c.shape[0])
        o.pml_outer, o.pml_iface = int(pml_outer), int(pml_iface)
        o.pml_power, o.pml_s0, o.pml_cref = float(pml_power), float(pml_s0), float(pml_cref)
        o.pml_iface_s0 = -1.0 if pml_iface_s0 is None else float(pml_iface_s0)
        o.beta_rule = int(beta_rule)
        o.sweep = {"double": 0, "concurrent": 1}[sweep]
        o.transmission = {"pml": 0, "robin": 1}[transmission]
        o.restart = int(restart)
        o.batch_fuse = 1 if batch_fuse else 0
        o.prec = {"c128": L.HELM_C128, "mixed": L.HELM_MIXED_C64, "c64": L.HELM_MIXED_C64}[prec]
        o.mode = {"full": L.HELM_FULL, "reduced": L.HELM_REDUCED}[mode]
        o.max_iter = int(max_iter)
        o.chunk = int(chunk)
        o.graph = 1 if graph else 0
        self._beta = None
        if beta is not None:
            self._beta = (ctypes.c_int * len(beta))(*[int(b) for b in beta])
            o.beta = ctypes.cast(self._beta, ctypes.POINTER(ctypes.c_int))
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            o.stream = ctypes.c_void_p(self.stream.cuda_stream)
            self._opts = o
            self.h = L.helm_setup(self._c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  omega, h, o, J)
        self.N_x, self.N_y, self.N_z, self.J = L.helm_get_dims3(self.h)
        self.dim = self._c.ndim
        self.row_shape = (self.N_z, self.N_y) if self.dim == 3 else (self.N_y,)
        self.beta, self.strip_first, self.strip_width = L.helm_get_partition(self.h, self.J)
        self.chunk_rows, self.n_chunks = L.helm_get_chunks(self.h)
        self.prec, self.mode = prec, mode
        self.omega, self.grid_h = float(omega), float(h)
        self.factored = False

    # ------------------------------------------------------------------ helpers
    def _field(self, x: torch.Tensor, name: str, cols: Optional[int] = None) -> torch.Tensor:
        cols = self.N_x if cols is None else cols
        if not isinstance(x, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if x.dtype != torch.complex128:
            raise TypeError(f"{name} must be complex128")
        if x.device != self.device:
            raise ValueError(f"{name} must live on {self.device}")
        want = self.row_shape + (cols,)
        if x.dim() == len(want):
            x = x.unsqueeze(0)
        if tuple(x.shape[1:]) != want:
            raise ValueError(f"{name} must have shape (nrhs, {', '.join(map(str, want))}), got {tuple(x.shape)}")
        return x.contiguous()

    def _sync(self):
        self.stream.synchronize()

    def _begin(self):
        """Order the handle's stream after the caller's current stream (inputs ready)."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _end(self):
        """Order the caller's current stream after the handle's work (outputs ready)."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    # ------------------------------------------------------------------ API
    def factor(self) -> "Helmholtz":
        self._begin()
        with torch.cuda.device(self.device):
            L.helm_factor(self.h)
        self._end()
        self.factored = True
        return self

    def autotune(self, rhs: torch.Tensor, candidates: Sequence[int] = (16, 24, 32, 40, 48),
                 reps: int = 2, cache: Optional[str] = "default") -> dict:
        """Pick the strip solver's rows per chunk by timing one GMRES iteration's operator
        on `rhs` for each candidate (helm_autotune); leaves the handle factored with the
        fastest.  Results are kept in a JSON cache keyed by the problem's shape (device
        name, precision, mode, padded grid, strip widths, right-hand sides): a hit skips the
        timing and only refactors with the cached choice.  cache=None disables it;
        "default" is $HELM_TUNE_CACHE or ~/.cache/paper_1208_3956_amd/tune.json."""
        from . import tune
        f = self._field(rhs, "rhs")
        key = tune.key(torch.cuda.get_device_name(self.device), self.prec, self.mode,
                       (self.N_x, self.N_y, self.N_z), self.strip_width, f.shape[0])
        path = tune.cache_path(cache)
        hit = tune.lookup(path, key) if path else None
        self._begin()
        with torch.cuda.device(self.device):
            if hit is not None:
                best, ms = L.helm_autotune(self.h, f.shape[0], f.data_ptr(), [int(hit)], 1)
                times = {}
            else:
                best, ms = L.helm_autotune(self.h, f.shape[0], f.data_ptr(), list(candidates), reps)
                times = {int(c): t for c, t in zip(candidates, ms)}
        self._end()
        if hit is None and path and self.dim == 2:
            tune.store(path, key, best, times)
        self.chunk_rows, self.n_chunks = L.helm_get_chunks(self.h)
        self.factored = True
        return {"chunk_rows": best, "ms_per_apply": times, "cached": hit is not None}

    @property
    def factor_slots(self) -> int:
        """Number of stored factorisations (identical 2-D strips share one)."""
        return L.helm_get_factor_slots(self.h, self.J)[0]

    @property
    def strip_factor_slot(self) -> list:
        """The factorisation slot of every strip."""
        return L.helm_get_factor_slots(self.h, self.J)[1]

    @property
    def factor_path(self) -> int:
        """3-D: 1 when the slab inverses came from the complex64 blocked Gauss-Jordan, 0
        when from the FP64 one (always 0 in 2-D)."""
        return L.helm_get_factor_path(self.h)

    def solve(self, rhs: torch.Tensor, tol: float = 1e-6) -> SolveResult:
        f = self._field(rhs, "rhs")
        u = torch.empty_like(f)
        self._begin()
        with torch.cuda.device(self.device):
            st, it, rel = L.helm_solve(self.h, f.shape[0], f.data_ptr(), u.data_ptr(), tol)
            ap, rs, ms = L.helm_get_stats(self.h)
            pr, prf = L.helm_get_panel_stats(self.h)
        self._end()
        return SolveResult(u, it, rel, st, ap, rs, ms, pr, prf)

    def grad(self, src: torch.Tensor, rec, d: torch.Tensor, tol: float = 1e-6):
        """Misfit 1/2 sum_s |R u_s - d_s|^2 and its gradient with respect to m = 1/c^2 on
        the interior grid (adjoint state, see helm_grad).  src: (nsrc, N_y, N_x) complex128;
        rec: flat padded-grid receiver indices (int64 tensor or sequence); d: (nsrc, nrec)
        complex128.  Returns (misfit, grad (n_y, n_x) float64 tensor, iterations)."""
        f = self._field(src, "src")
        nsrc = f.shape[0]
        rec_t = torch.as_tensor(rec, dtype=torch.int64).to(self.device).contiguous().reshape(-1)
        nrec = rec_t.numel()
        if not isinstance(d, torch.Tensor) or d.dtype != torch.complex128 or d.device != self.device:
            raise TypeError("d must be a complex128 tensor on the solver's device")
        if tuple(d.shape) != (nsrc, nrec):
            raise ValueError(f"d must have shape ({nsrc}, {nrec}), got {tuple(d.shape)}")
        d = d.contiguous()
        if self.dim != 2:
            raise ValueError("the gradient is provided for 2-D problems")
        n_y, n_x = self._c.shape
        g = torch.empty((n_y, n_x), dtype=torch.float64, device=self.device)
        self._begin()
        with torch.cuda.device(self.device):
            st, mis, its = L.helm_grad(self.h, nsrc, f.data_ptr(), nrec, rec_t.data_ptr(), d.data_ptr(),
                                       tol, g.data_ptr())
        self._end()
        return mis, g, its

    def apply_P(self, f: torch.Tensor) -> torch.Tensor:
        f = self._field(f, "f")
        out = torch.empty_like(f)
        self._begin()
        with torch.cuda.device(self.device):
            L.helm_apply_P(self.h, f.shape[0], f.data_ptr(), out.data_ptr())
        self._end()
        return out

    def apply_AP_reduced(self, psi: torch.Tensor) -> torch.Tensor:
        psi = self._field(psi, "psi", cols=2 * (self.J - 1))
        out = torch.empty_like(psi)
        self._begin()
        with torch.cuda.device(self.device):
            L.helm_apply_AP_reduced(self.h, psi.shape[0], psi.data_ptr(), out.data_ptr())
        self._end()
        return out

    def restart_rhs_reduced(self, r: torch.Tensor) -> torch.Tensor:
        """(r - A P r) on the reduced columns, from the target-only sweeps (helm_restart_rhs_reduced)."""
        r = self._field(r, "r")
        out = torch.empty((r.shape[0],) + tuple(r.shape[1:-1]) + (2 * (self.J - 1),), dtype=r.dtype,
                          device=r.device)
        self._begin()
        with torch.cuda.device(self.device):
            L.helm_restart_rhs_reduced(self.h, r.shape[0], r.data_ptr(), out.data_ptr())
        self._end()
        return out

    def apply_A(self, u: torch.Tensor, f: Optional[torch.Tensor] = None) -> torch.Tensor:
        u = self._field(u, "u")
        if f is not None:
            f = self._field(f, "f")
            if f.shape != u.shape:
                raise ValueError("u and f must have the same shape")
        out = torch.empty_like(u)
        self._begin()
        with torch.cuda.device(self.device):
            L.helm_apply_A(self.h, u.shape[0], u.data_ptr(), f.data_ptr() if f is not None else 0,
                           out.data_ptr())
        self._end()
        return out

    def strip_solve(self, strip: int, r: torch.Tensor) -> torch.Tensor:
        if not 0 <= strip < self.J:
            raise ValueError("strip out of range")
        r = self._field(r, "r", cols=self.strip_width[strip])
        x = torch.empty_like(r)
        self._begin()
        with torch.cuda.device(self.device):
            L.helm_strip_solve(self.h, strip, r.shape[0], r.data_ptr(), x.data_ptr())
        self._end()
        return x

    def set_kernel_timing(self, enable=True, classes=None):
        """Bracket hot-kernel launches with HIP events (see helm_set_kernel_timing): all
        classes, or only those named in `classes` (names as in kernel_times())."""
        mask = 0
        if enable:
            mask = 0xFF if classes is None else sum(1 << L.KERNEL_CLASSES.index(c) for c in classes)
        L.helm_set_kernel_timing(self.h, mask)

    def kernel_times(self) -> dict:
        """{class: (launches, total ms)} since timing was enabled."""
        return L.helm_get_kernel_times(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            L.helm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def solve_batch(problems: Sequence[Helmholtz], rhs: Sequence[torch.Tensor], tol: float = 1e-6):
    """Solve several independent problems concurrently (helm_solve_batch): one host thread
    per problem, each on its handle's stream.  Returns one SolveResult per problem."""
    if len(problems) != len(rhs) or not problems:
        raise ValueError("one right-hand-side tensor per problem is required")
    fs = [H._field(f, "rhs") for H, f in zip(problems, rhs)]
    us = [torch.empty_like(f) for f in fs]
    for H in problems:
        torch.cuda.current_stream(H.device).synchronize()   # inputs ready before other streams read them
    nr = [f.shape[0] for f in fs]
    st, its, rel = L.helm_solve_batch([H.h for H in problems], nr, [f.data_ptr() for f in fs],
                                      [u.data_ptr() for u in us], tol)
    out, k = [], 0
    for H, u, n in zip(problems, us, nr):
        H.stream.synchronize()
        ap, rs, ms = L.helm_get_stats(H.h)
        pr, prf = L.helm_get_panel_stats(H.h)
        fu, un = L.helm_get_fusion_stats(H.h)
        out.append(SolveResult(u, its[k:k + n], rel[k:k + n], st, ap, rs, ms, pr, prf, fu, un))
        k += n
    return out
