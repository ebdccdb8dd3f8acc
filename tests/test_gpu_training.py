"""Synthetic end-to-end training through the PF layer (both completion
steps, implicit adjoint): the loss falls, every scenario keeps converging,
and the gradient reaching the decision block matches the oracle's."""
import numpy as np
import pytest

from gen.grids import make_case
from oracle.completion import adjoint_completed, recover
from oracle.newton import newton
from oracle.ybus import ybus_of

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,batch,precision", [("c1", 256, "mixed"), ("c3", 128, "fp64")])
def test_training_loss_falls_and_scenarios_converge(name, batch, precision, device):
    import torch
    from paper_2606_07099_amd.training import SyntheticDispatchTask
    spec, net, sc = make_case(name, batch=batch)
    task = SyntheticDispatchTask(net, sc, device, precision=precision, tol=spec.tol, lr=3e-3)
    losses = [float(task.step()) for _ in range(30)]
    torch.cuda.synchronize()
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.98 * losses[0], losses
    vm, va, iters, status, fn = task.tpl.solve(task.pd, task.qd, task.pg0, task.vset0)
    assert int((status != 0).sum()) == 0


def test_training_gradient_of_the_decision_block_matches_oracle(device):
    """One forward/backward of the task's loss: dL/d(pg, vset) through the
    layer against the oracle's completed adjoint at the oracle's solution."""
    import torch
    from paper_2606_07099_amd.training import SyntheticDispatchTask
    spec, net, sc = make_case("c1", batch=32)
    task = SyntheticDispatchTask(net, sc, device, precision="fp64", tol=1e-10)
    pg = task.pg0.clone().requires_grad_(True)
    vset = task.vset0.clone().requires_grad_(True)
    vm, va, po, qo = task.layer(task.pd, task.qd, pg, vset)
    gen_p = po * task.gen_w
    L = ((task.c2 * gen_p ** 2 + task.c1 * gen_p).sum()
         + task.v_weight * (torch.relu(vm - 1.05) ** 2 + torch.relu(0.95 - vm) ** 2).sum()
         + task.q_weight * ((qo * task.gen_w) ** 2).sum())
    L.backward()
    Y = ybus_of(net)
    bt = net.bus_type
    gw = (bt != 0).astype(float)
    for b in (0, 13, 31):
        r = newton(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=1e-10)
        rp, rq = recover(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], r.vm, r.va)
        g_vm = task.v_weight * (2 * np.maximum(r.vm - 1.05, 0) - 2 * np.maximum(0.95 - r.vm, 0))
        g_po = (2 * task.c2 * rp + task.c1) * gw
        g_qo = 2 * task.q_weight * rq * gw
        g = adjoint_completed(Y, bt, r.vm, r.va, g_vm, np.zeros_like(r.va), g_po, g_qo)
        for ours, ref in ((pg.grad[b].cpu().numpy(), g.pg), (vset.grad[b].cpu().numpy(), g.vset)):
            assert np.linalg.norm(ours - ref) <= 1e-6 * max(np.linalg.norm(ref), 1e-12), b
