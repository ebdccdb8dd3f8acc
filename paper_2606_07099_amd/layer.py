"""Implicit power-flow layer for PyTorch autograd.

Forward: batched Newton completion of (|V|, theta) from the loads and the
decision block (p_g on PV buses, |V| setpoints on PV and slack buses)
(forward pass with equality completion, Sec. II-B).  Backward: implicit
differentiation through the converged LU factors, J1^T lambda = g_z1 and
the J3 term (backward pass, Sec. II-B), all inside the HIP library.
"""
from __future__ import annotations

import torch

from .pf import PFTemplate


class PFLayerFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tpl: PFTemplate, pd, qd, pg, vset):
        vm, va, iters, status, fn = tpl.solve(pd.contiguous(), qd.contiguous(), pg.contiguous(),
                                              vset.contiguous())
        ctx.tpl = tpl
        ctx.solve_id = tpl._solve_id
        ctx.aux = (iters, status, fn)
        return vm, va

    @staticmethod
    def backward(ctx, g_vm, g_va):
        tpl = ctx.tpl
        if tpl._solve_id != ctx.solve_id:
            raise RuntimeError("PFLayer: the template was used for another solve before backward; "
                               "use one template per pending forward")
        ref = g_vm if g_vm is not None else g_va
        g_vm = torch.zeros_like(ref) if g_vm is None else g_vm.contiguous()
        g_va = torch.zeros_like(ref) if g_va is None else g_va.contiguous()
        g_pd, g_qd, g_pg, g_vset = tpl.adjoint(g_vm, g_va)
        return None, g_pd, g_qd, g_pg, g_vset


class PFLayer(torch.nn.Module):
    """``vm, va = PFLayer(template)(pd, qd, pg, vset)``; the per-scenario
    Newton outcome of the last call is in ``.last_status`` / ``.last_iters``
    / ``.last_mismatch``."""

    def __init__(self, template: PFTemplate):
        super().__init__()
        self.template = template
        self.last_iters = self.last_status = self.last_mismatch = None

    def forward(self, pd, qd, pg, vset):
        vm, va = PFLayerFunction.apply(self.template, pd, qd, pg, vset)
        return vm, va
