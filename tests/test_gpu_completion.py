"""GPU Step-2 recovery and the adjoint of the full two-step completion
(Sec. II-B: eq. F2_completion, the chain-rule, J2 and vbar2 equations)
against the oracle, through the C ABI and through the autograd layer."""
import numpy as np
import pytest

from gpu_helpers import make_gpu_case, random_states, to_dev
from oracle.adjoint import adjoint, loss, loss_grad, solve_polished
from oracle.completion import (adjoint_completed, generation_loss, generation_loss_grad,
                               recover, recover_batch)
from oracle.newton import Index, newton
from oracle.ybus import ybus_of

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)


@pytest.mark.parametrize("name,batch", [("c0", 64), ("c3", 40), ("c2", 24)])
def test_recover_matches_oracle_at_random_states(name, batch, device):
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, batch=batch)
    vm, va = random_states(net, batch, seed=11)
    po, qo = tpl.recover(d["pd"], d["qd"], d["pg"], to_dev(vm, device), to_dev(va, device))
    torch.cuda.synchronize()
    po, qo = po.cpu().numpy(), qo.cpu().numpy()
    rp, rq = recover_batch(ybus_of(net), net.bus_type, sc.pd, sc.qd, sc.pg, vm, va)
    bt = net.bus_type
    # one Y_bus row product per entry in FP64: summation order only
    scale = np.abs(ybus_of(net)).sum(axis=1).max()
    assert np.abs(po - rp).max() <= 1e-13 * scale * 4
    assert np.abs(qo - rq).max() <= 1e-13 * scale * 4
    # exact pass-through on PV buses and exact zeros on PQ buses
    assert np.array_equal(po[:, bt == 1], sc.pg[:, bt == 1])
    assert np.all(po[:, bt == 0] == 0.0) and np.all(qo[:, bt == 0] == 0.0)


def test_recover_without_pg_and_with_null_outputs(device):
    import torch
    from paper_2606_07099_amd._lib import lib, check
    import ctypes
    spec, net, sc, tpl, d, tol = make_gpu_case("c0", device, batch=8)
    vm, va = random_states(net, 8, seed=3)
    vm_d, va_d = to_dev(vm, device), to_dev(va, device)
    po, qo = tpl.recover(d["pd"], d["qd"], None, vm_d, va_d)
    torch.cuda.synchronize()
    rp, rq = recover_batch(ybus_of(net), net.bus_type, sc.pd, sc.qd, np.zeros_like(sc.pg), vm, va)
    assert np.abs(po.cpu().numpy() - rp).max() < 1e-11
    assert np.abs(qo.cpu().numpy() - rq).max() < 1e-11
    q2 = torch.full_like(vm_d, 7.0)
    check(lib().pf_recover_batch(tpl._h, ctypes.c_void_p(d["pd"].data_ptr()),
                                 ctypes.c_void_p(d["qd"].data_ptr()), ctypes.c_void_p(0),
                                 ctypes.c_void_p(vm_d.data_ptr()), ctypes.c_void_p(va_d.data_ptr()),
                                 ctypes.c_void_p(0), ctypes.c_void_p(q2.data_ptr()), ctypes.c_void_p(0)))
    torch.cuda.synchronize()
    assert torch.equal(q2, qo)


@pytest.mark.parametrize("name,precision,n_check", [("c0", "fp64", 64), ("c3", "fp64", 8),
                                                    ("c1", "mixed", 16), ("c3", "mixed", 8),
                                                    ("c2", "mixed", 3)])
def test_completed_adjoint_matches_dense_oracle(name, precision, n_check, device):
    import torch
    batch = 256 if name == "c2" else None
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, precision=precision, batch=batch)
    bt = net.bus_type
    vm, va, iters, status, fn = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    po, qo = tpl.recover(d["pd"], d["qd"], d["pg"], vm, va)
    g_vm, g_va = loss_grad(vm.cpu().numpy(), va.cpu().numpy())
    g_po, g_qo = generation_loss_grad(po.cpu().numpy(), qo.cpu().numpy(), bt)
    outs = tpl.adjoint_completed(to_dev(g_vm, device), to_dev(g_va, device), to_dev(g_po, device),
                                 to_dev(g_qo, device))
    plain = tpl.adjoint(to_dev(g_vm, device), to_dev(g_va, device))
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)
    g_pd, g_qd, g_pg, g_vs = [o.cpu().numpy() for o in outs]
    Y = ybus_of(net)
    for b in np.unique(np.linspace(0, sc.batch - 1, n_check).astype(int)):
        r = newton(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=tol)
        rp, rq = recover(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], r.vm, r.va)
        gv, ga = loss_grad(r.vm, r.va)
        gp, gq = generation_loss_grad(rp, rq, bt)
        g = adjoint_completed(Y, bt, r.vm, r.va, gv, ga, gp, gq)
        ours = np.concatenate([g_pd[b], g_qd[b], g_pg[b], g_vs[b]])
        ref = np.concatenate([g.pd, g.qd, g.pg, g.vset])
        assert _rel(ours, ref) <= 1e-6, (b, _rel(ours, ref))
        assert np.all(g_pg[b][bt != 1] == 0.0) and np.all(g_vs[b][bt == 0] == 0.0)
    # the generation terms change the answer; without them it is pf_adjoint_batch
    none = tpl.adjoint_completed(to_dev(g_vm, device), to_dev(g_va, device))
    torch.cuda.synchronize()
    for a, p in zip(none, plain):
        assert torch.equal(a, p)
    assert not np.allclose(g_pd, plain[0].cpu().numpy())


def test_completed_adjoint_matches_central_differences(device):
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case("c0", device, batch=4, tol=1e-12)
    bt = net.bus_type
    vm, va, iters, status, fn = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    po, qo = tpl.recover(d["pd"], d["qd"], d["pg"], vm, va)
    g_vm, g_va = loss_grad(vm.cpu().numpy(), va.cpu().numpy())
    g_po, g_qo = generation_loss_grad(po.cpu().numpy(), qo.cpu().numpy(), bt)
    outs = tpl.adjoint_completed(*(to_dev(a, device) for a in (g_vm, g_va, g_po, g_qo)))
    torch.cuda.synchronize()
    ours = dict(zip(("pd", "qd", "pg", "vset"), (o.cpu().numpy() for o in outs)))
    Y = ybus_of(net)
    idx = Index.of(bt)
    n = net.n_bus

    def total(a):
        v, t = solve_polished(Y, bt, a["pd"], a["qd"], a["pg"], a["vset"])
        p, q = recover(Y, bt, a["pd"], a["qd"], a["pg"], v, t)
        return loss(v, t) + generation_loss(p, q, bt)

    h = 1e-6
    for b in range(2):
        args = {"pd": sc.pd[b], "qd": sc.qd[b], "pg": sc.pg[b], "vset": sc.vset[b]}
        for which, coords in (("pd", np.arange(n)), ("qd", np.arange(n)), ("pg", idx.pv),
                              ("vset", np.concatenate([idx.pv, idx.ref]))):
            fd = np.zeros(len(coords))
            for c, j in enumerate(coords):
                vals = []
                for s in (+1.0, -1.0):
                    a = {k: v.copy() for k, v in args.items()}
                    a[which][j] += s * h
                    vals.append(total(a))
                fd[c] = (vals[0] - vals[1]) / (2 * h)
            assert _rel(ours[which][b][coords], fd) <= 1e-6, (which, b)


def test_completed_layer_autograd_end_to_end(device):
    import torch
    from paper_2606_07099_amd import PFLayer
    spec, net, sc, tpl, d, tol = make_gpu_case("c3", device, batch=64, tol=1e-10)
    bt = net.bus_type
    layer = PFLayer(tpl, recover=True)
    leaves = {k: d[k].clone().requires_grad_(True) for k in ("pd", "qd", "pg", "vset")}
    vm, va, po, qo = layer(leaves["pd"], leaves["qd"], leaves["pg"], leaves["vset"])
    slack = torch.as_tensor(bt == 2, device=device)
    gen = torch.as_tensor(bt != 0, device=device)
    L = ((torch.relu(vm - 1.05) ** 2).sum() + (torch.relu(0.95 - vm) ** 2).sum() + 0.1 * (va ** 2).sum()
         + (po[:, slack] ** 2).sum() + 0.5 * (qo[:, gen] ** 2).sum())
    L.backward()
    Y = ybus_of(net)
    for b in (0, 31, 63):
        r = newton(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=1e-10)
        rp, rq = recover(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], r.vm, r.va)
        assert np.abs(po[b].detach().cpu().numpy() - rp).max() < 1e-6
        assert np.abs(qo[b].detach().cpu().numpy() - rq).max() < 1e-6
        gv, ga = loss_grad(r.vm, r.va)
        gp, gq = generation_loss_grad(rp, rq, bt)
        g = adjoint_completed(Y, bt, r.vm, r.va, gv, ga, gp, gq)
        for k in ("pd", "qd", "pg", "vset"):
            assert _rel(leaves[k].grad[b].cpu().numpy(), getattr(g, k)) <= 1e-6, (k, b)


@pytest.mark.parametrize("precision,batch", [("fp64", 1024), ("mixed", 1024), ("mixed", 200)])
def test_hbm_resident_slices_on_the_118_bus_grid(precision, batch, device):
    """The 118-bus grid forced onto HBM-resident slices (1024 threads; slice
    width 2 at batch 1024, 1 at batch 200, with a ragged last slice): the
    same solution and gradients as the oracle, through both completion steps."""
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case("c1", device, precision=precision, batch=batch,
                                               block_threads=1024)
    info = tpl.info()
    assert info["lds_resident"] == 0 and info["block_threads"] == 1024
    bt = net.bus_type
    vm, va, iters, status, fn = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    po, qo = tpl.recover(d["pd"], d["qd"], d["pg"], vm, va)
    g_vm, g_va = loss_grad(vm.cpu().numpy(), va.cpu().numpy())
    g_po, g_qo = generation_loss_grad(po.cpu().numpy(), qo.cpu().numpy(), bt)
    outs = tpl.adjoint_completed(*(to_dev(a, device) for a in (g_vm, g_va, g_po, g_qo)))
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)
    vm, va, iters = vm.cpu().numpy(), va.cpu().numpy(), iters.cpu().numpy()
    grads = [o.cpu().numpy() for o in outs]
    Y = ybus_of(net)
    for b in np.unique(np.linspace(0, batch - 1, 12).astype(int)):
        r = newton(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=tol)
        assert np.abs(vm[b] - r.vm).max() <= 1e-8 and np.abs(va[b] - r.va).max() <= 1e-8
        assert iters[b] - r.iters in ((0,) if precision == "fp64" else (0, 1))
        rp, rq = recover(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], r.vm, r.va)
        gv, ga = loss_grad(r.vm, r.va)
        gp, gq = generation_loss_grad(rp, rq, bt)
        g = adjoint_completed(Y, bt, r.vm, r.va, gv, ga, gp, gq)
        ours = np.concatenate([x[b] for x in grads])
        ref = np.concatenate([g.pd, g.qd, g.pg, g.vset])
        assert _rel(ours, ref) <= 1e-6, b
