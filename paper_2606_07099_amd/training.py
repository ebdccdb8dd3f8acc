"""Synthetic end-to-end training through the PF layer: the analogue of the
paper's layer-training experiments (Sec. IV-C, Tables V and VI), with a
synthetic task in place of the DC3 and DeepLDE models and their datasets.

A small MLP maps each scenario's loads to the decision block x (eq. ynn):
the PV dispatch and the |V| setpoints on PV and slack buses, as bounded
corrections of a nominal operating point.  The PF layer completes the state
by both completion steps (Newton for z1, Step-2 recovery of z2) and the loss
is a quadratic generation cost over every generator (the slack's output is
the recovered p_g,R) plus voltage-band and reactive-output penalties.  The
backward pass runs the implicit adjoint of the layer.  Every step of the
layer runs in the HIP library; the MLP, the loss and the optimizer are plain
torch.
"""
from __future__ import annotations

import numpy as np
import torch

from .layer import PFLayer
from .pf import PFTemplate


class DispatchMLP(torch.nn.Module):
    """Loads (P and Q of the PQ buses, relative to nominal) -> relative
    dispatch corrections on PV buses and |V| setpoint corrections on PV and
    slack buses, both bounded by tanh."""

    def __init__(self, n_in: int, n_pv: int, n_gen: int, hidden: int = 256,
                 dp_max: float = 0.1, dv_max: float = 0.03):
        super().__init__()
        self.n_pv = n_pv
        self.dp_max, self.dv_max = dp_max, dv_max
        self.net = torch.nn.Sequential(
            torch.nn.Linear(n_in, hidden), torch.nn.ReLU(),
            torch.nn.Linear(hidden, hidden), torch.nn.ReLU(),
            torch.nn.Linear(hidden, n_pv + n_gen))
        # start at the nominal operating point
        torch.nn.init.zeros_(self.net[-1].weight)
        torch.nn.init.zeros_(self.net[-1].bias)

    def forward(self, u):
        o = self.net(u)
        return (self.dp_max * torch.tanh(o[:, :self.n_pv]),
                self.dv_max * torch.tanh(o[:, self.n_pv:]))


class SyntheticDispatchTask:
    """One network and a fixed batch of load scenarios; ``step()`` is one
    optimizer step over the whole batch."""

    def __init__(self, net, scenarios, device, *, precision: str = "mixed", tol: float = 1e-8,
                 hidden: int = 256, lr: float = 1e-3, seed: int = 0,
                 cost=(1.0, 0.1), v_weight: float = 10.0, q_weight: float = 0.1):
        torch.manual_seed(seed)
        bt = np.asarray(net.bus_type)
        self.batch = scenarios.batch
        self.n_bus = net.n_bus
        self.tpl = PFTemplate.from_network(net, self.batch, tol=tol, precision=precision,
                                           keep_factors=True)
        self.layer = PFLayer(self.tpl, recover=True)
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.pd = torch.as_tensor(scenarios.pd, **f64)
        self.qd = torch.as_tensor(scenarios.qd, **f64)
        self.pg0 = torch.as_tensor(scenarios.pg, **f64)
        self.vset0 = torch.as_tensor(scenarios.vset, **f64)
        pq = np.flatnonzero(bt == 0)
        self.pv = torch.as_tensor(np.flatnonzero(bt == 1), device=dev)
        self.gen = torch.as_tensor(np.flatnonzero(bt != 0), device=dev)
        self.gen_w = torch.as_tensor((bt != 0).astype(np.float64), **f64)
        p_nom = np.maximum(np.asarray(net.p0)[pq], 1e-6)
        q_nom = np.where(np.abs(np.asarray(net.q0)[pq]) > 1e-6, np.asarray(net.q0)[pq], 1.0)
        u = np.concatenate([scenarios.pd[:, pq] / p_nom, scenarios.qd[:, pq] / q_nom], axis=1)
        self.u = torch.as_tensor(u, dtype=torch.float32, device=dev)
        self.model = DispatchMLP(u.shape[1], int(self.pv.numel()), int(self.gen.numel()),
                                 hidden).to(dev)
        self.opt = torch.optim.Adam(self.model.parameters(), lr=lr)
        self.c2, self.c1 = cost
        self.v_weight, self.q_weight = v_weight, q_weight

    def forward_loss(self):
        dp, dv = self.model(self.u)
        zeros = torch.zeros_like(self.pg0)
        pg = self.pg0 * (1.0 + zeros.index_add(1, self.pv, dp.double()))
        vset = self.vset0 + zeros.index_add(1, self.gen, dv.double())
        vm, va, po, qo = self.layer(self.pd, self.qd, pg, vset)
        # every generator's active output: x's dispatch on PV buses and the
        # recovered p_g on the slack bus (pg_out holds both)
        gen_p = po * self.gen_w
        cost = (self.c2 * gen_p ** 2 + self.c1 * gen_p).sum(dim=1)
        band = (torch.relu(vm - 1.05) ** 2 + torch.relu(0.95 - vm) ** 2).sum(dim=1)
        reactive = ((qo * self.gen_w) ** 2).sum(dim=1)
        return (cost + self.v_weight * band + self.q_weight * reactive).mean()

    def step(self) -> torch.Tensor:
        self.opt.zero_grad(set_to_none=True)
        loss = self.forward_loss()
        loss.backward()
        self.opt.step()
        return loss.detach()
