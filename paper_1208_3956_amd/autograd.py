"""torch.autograd interface of the misfit: J(m) = 1/2 sum_s |R u_s(m) - d_s|^2 with
A(m) u_s = f_s and m = 1/c^2 on the interior grid.

forward() sets up and factors the problem for the given m (every call; the factors depend
on m) and evaluates J and dJ/dm in one helm_grad call; backward() returns
grad_output * dJ/dm.  The PML is part of the fixed problem: its reference speed `pml_cref`
must be given, so that it does not move with m.
"""
from __future__ import annotations

import torch

from .solver import Helmholtz


class HelmMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m: torch.Tensor, src: torch.Tensor, rec: torch.Tensor, d: torch.Tensor,
                cfg: dict) -> torch.Tensor:
        if m.dtype != torch.float64 or m.dim() != 2:
            raise TypeError("m must be a 2-D float64 tensor (n_y, n_x)")
        if not (m > 0).all():
            raise ValueError("m = 1/c^2 must be positive")
        if not cfg.get("pml_cref"):
            raise ValueError("cfg['pml_cref'] must fix the PML reference speed")
        c = (1.0 / torch.sqrt(m.detach())).cpu().numpy()
        H = Helmholtz(c, cfg["omega"], cfg["h"], cfg["J"], cfg.get("pml_outer", 16),
                      cfg.get("pml_iface", 8), cfg.get("pml_power", 2.0), cfg.get("pml_s0", 10.0),
                      pml_cref=cfg["pml_cref"], pml_iface_s0=cfg.get("pml_iface_s0"),
                      prec=cfg.get("prec", "c128"),
                      mode=cfg.get("mode", "full"), chunk=cfg.get("chunk", 0), device=src.device)
        try:
            H.factor()
            mis, g, _ = H.grad(src, rec, d, cfg.get("tol", 1e-8))
        finally:
            H.close()
        ctx.save_for_backward(g.to(m.device))
        return torch.tensor(mis, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None


def misfit(m: torch.Tensor, src: torch.Tensor, rec, d: torch.Tensor, **cfg) -> torch.Tensor:
    """J(m) as a differentiable scalar; cfg: omega, h, J, pml_cref (required), pml_outer,
    pml_iface, pml_power, pml_s0, pml_iface_s0, prec, mode, chunk, tol."""
    return HelmMisfit.apply(m, src, torch.as_tensor(rec, dtype=torch.int64), d, cfg)
