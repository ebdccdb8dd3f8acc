"""Shared set-up of the GPU tests: seeded cases, device tensors, oracle
references.  The oracle and the HIP path only share the generated inputs."""
from __future__ import annotations

import numpy as np

from gen.grids import SPECS, make_case
from oracle.newton import Index, newton, newton_batch, j1, mismatch, specified
from oracle.ybus import ybus_of


def to_dev(a, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)


def make_gpu_case(name, device, batch=None, precision="fp64", tol=None, max_iter=20,
                  keep_factors=True, scenario_mode="lognormal", **kw):
    from paper_2606_07099_amd import PFTemplate
    spec, net, sc = make_case(name, batch=batch, scenario_mode=scenario_mode)
    tol = spec.tol if tol is None else tol
    tpl = PFTemplate.from_network(net, sc.batch, tol=tol, max_iter=max_iter, precision=precision,
                                  keep_factors=keep_factors, **kw)
    dev = {k: to_dev(getattr(sc, k), device) for k in ("pd", "qd", "pg", "vset")}
    return spec, net, sc, tpl, dev, tol


def paper_col_perm(net):
    """Column permutation from the oracle's unknown order (theta_(B\\R), |V|_D)
    to the paper's order (|V|_D, theta_(B\\R))."""
    idx = Index.of(net.bus_type)
    npvpq, npq = idx.pvpq.size, idx.pq.size
    return np.concatenate([np.arange(npvpq, npvpq + npq), np.arange(npvpq)])


def oracle_j1_paper(net, vm, va):
    J = j1(ybus_of(net), vm * np.exp(1j * va), Index.of(net.bus_type))
    return J[:, paper_col_perm(net)]


def oracle_f1(net, sc, b, vm, va):
    p, q = specified(sc.pd[b], sc.qd[b], sc.pg[b], net.bus_type)
    return mismatch(ybus_of(net), vm * np.exp(1j * va), p, q, Index.of(net.bus_type))


def random_states(net, count, seed):
    rng = np.random.default_rng(seed)
    vm = rng.uniform(0.92, 1.08, (count, net.n_bus))
    va = rng.uniform(-0.3, 0.3, (count, net.n_bus))
    slack = net.bus_type == 2
    va[:, slack] = 0.0
    return vm, va


def tie_band(history, iters_gpu, iters_or, tol):
    """True when the two iteration counts differ only because ||F1|| sat
    within 1e-3 tol of the tolerance at the deciding iteration."""
    t = min(iters_gpu, iters_or)
    return t < len(history) and abs(history[t] - tol) < 1e-3 * tol
