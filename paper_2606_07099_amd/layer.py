"""Implicit power-flow layer for PyTorch autograd.

Forward: batched Newton completion of (|V|, theta) from the loads and the
decision block (p_g on PV buses, |V| setpoints on PV and slack buses)
(forward pass with equality completion, Sec. II-B, Step 1), optionally
followed by the explicit recovery of the generation block (Step 2).
Backward: implicit differentiation through the converged LU factors,
J1^T lambda = g_z1 and the J3 term, plus vbar2 = -J2^T dL/dz2 when the
generation block is an output (backward pass, Sec. II-B), all inside the HIP
library.
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


class PFCompletedLayerFunction(torch.autograd.Function):
    """Both completion steps: outputs (vm, va, pg_out, qg_out)."""

    @staticmethod
    def forward(ctx, tpl: PFTemplate, pd, qd, pg, vset):
        pd, qd, pg = pd.contiguous(), qd.contiguous(), pg.contiguous()
        vm, va, iters, status, fn = tpl.solve(pd, qd, pg, vset.contiguous())
        pg_out, qg_out = tpl.recover(pd, qd, pg, vm, va)
        ctx.tpl = tpl
        ctx.solve_id = tpl._solve_id
        ctx.aux = (iters, status, fn)
        return vm, va, pg_out, qg_out

    @staticmethod
    def backward(ctx, g_vm, g_va, g_pgo, g_qgo):
        tpl = ctx.tpl
        if tpl._solve_id != ctx.solve_id:
            raise RuntimeError("PFLayer: the template was used for another solve before backward; "
                               "use one template per pending forward")
        ref = next(g for g in (g_vm, g_va, g_pgo, g_qgo) if g is not None)
        g_vm = torch.zeros_like(ref) if g_vm is None else g_vm.contiguous()
        g_va = torch.zeros_like(ref) if g_va is None else g_va.contiguous()
        g_pgo = None if g_pgo is None else g_pgo.contiguous()
        g_qgo = None if g_qgo is None else g_qgo.contiguous()
        g_pd, g_qd, g_pg, g_vset = tpl.adjoint_completed(g_vm, g_va, g_pgo, g_qgo)
        return None, g_pd, g_qd, g_pg, g_vset


class PFLayer(torch.nn.Module):
    """``vm, va = PFLayer(template)(pd, qd, pg, vset)``; with
    ``recover=True`` the layer also returns the Step-2 generation block:
    ``vm, va, pg_out, qg_out``."""

    def __init__(self, template: PFTemplate, recover: bool = False):
        super().__init__()
        self.template = template
        self.recover = recover

    def forward(self, pd, qd, pg, vset):
        if self.recover:
            return PFCompletedLayerFunction.apply(self.template, pd, qd, pg, vset)
        vm, va = PFLayerFunction.apply(self.template, pd, qd, pg, vset)
        return vm, va
