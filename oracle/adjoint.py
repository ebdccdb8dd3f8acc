"""Implicit-differentiation gradients of the Step-1 completion (Sec. II-B,
backward pass), dense and one scenario at a time.

At the converged z1*, with g_z1 = dL/dz1 and J1 = dF1/dz1, the paper solves
J1^T lambda = g_z1^T and forms dL/dx = g_x - [lambda_G ; J3^T lambda] with
J3 = dF1/d|V|_(B\\D) (chain rule and the J3 equation of Sec. II-B).  Here the
dense calculated-injection Jacobian Jc = -J1 is used, so lambda = -mu with
Jc^T mu = g_z1, and the gradients read:

* loads (the scenario data u; dF1/dp_d = -I on the dP rows):
  dL/dp_d,i = lambda_P,i = -mu_P,i on non-slack buses, dL/dq_d,i = -mu_Q,i on
  PQ buses, zero elsewhere (those entries only move the Step-2 outputs);
* PV dispatch (x block, dF1/dp_g = +I on the dP rows): dL/dp_g,i = +mu_P,i;
* |V| setpoints (x block): dL/dV_set,j = dL/d|V|_j (direct pass-through)
  - sum_r mu_r d(calc_r)/d|V|_j for j in PV and slack, with the column
  taken from the full dense dS/d|V|.

The training loss is the one of the differentiable-layer workload:
L = sum over scenarios and buses of relu(|V|-1.05)^2 + relu(0.95-|V|)^2 plus
0.1 * sum theta^2 (angles in radians, slack angle fixed at 0).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .newton import Index, dS_dV, jacobian_calc, newton, CONVERGED, MAX_ITER


def loss(vm: np.ndarray, va: np.ndarray) -> float:
    over = np.maximum(vm - 1.05, 0.0)
    under = np.maximum(0.95 - vm, 0.0)
    return float(np.sum(over ** 2) + np.sum(under ** 2) + 0.1 * np.sum(va ** 2))


def loss_grad(vm: np.ndarray, va: np.ndarray):
    """(dL/d|V|, dL/dtheta) of :func:`loss`."""
    g_vm = 2.0 * np.maximum(vm - 1.05, 0.0) - 2.0 * np.maximum(0.95 - vm, 0.0)
    g_va = 0.2 * va
    return g_vm, g_va


@dataclass
class Grad:
    pd: np.ndarray
    qd: np.ndarray
    pg: np.ndarray
    vset: np.ndarray
    lam: np.ndarray      # the paper's lambda in (theta_(B\R), |V|_D) order


def adjoint(Y, bus_type, vm, va, g_vm, g_va) -> Grad:
    """Gradients w.r.t. (p_d, q_d, p_g, V_set) for ONE converged scenario."""
    idx = Index.of(bus_type)
    n = len(bus_type)
    V = vm * np.exp(1j * va)
    Jc = jacobian_calc(Y, V, idx)
    g_z1 = np.concatenate([g_va[idx.pvpq], g_vm[idx.pq]])
    mu = np.linalg.solve(Jc.T, g_z1)
    npvpq = idx.pvpq.size
    mu_p = np.zeros(n)
    mu_q = np.zeros(n)
    mu_p[idx.pvpq] = mu[:npvpq]
    mu_q[idx.pq] = mu[npvpq:]
    g_pd = -mu_p
    g_qd = -mu_q
    g_pg = np.zeros(n)
    g_pg[idx.pv] = mu_p[idx.pv]
    _, dVm = dS_dV(Y, V)
    g_vset = np.zeros(n)
    for j in np.concatenate([idx.pv, idx.ref]):
        col = np.concatenate([dVm[idx.pvpq, j].real, dVm[idx.pq, j].imag])
        g_vset[j] = g_vm[j] - mu @ col
    return Grad(g_pd, g_qd, g_pg, g_vset, -mu)


def adjoint_batch(Y, bus_type, vm, va, g_vm, g_va) -> Grad:
    out = [adjoint(Y, bus_type, vm[b], va[b], g_vm[b], g_va[b]) for b in range(vm.shape[0])]
    return Grad(*(np.stack([getattr(o, k) for o in out]) for k in ("pd", "qd", "pg", "vset", "lam")))


def solve_polished(Y, bus_type, pd, qd, pg, vset):
    """Forward solve driven to the rounding floor (for finite differences):
    tolerance 1e-13, accepted when it stagnates below 1e-11."""
    r = newton(Y, bus_type, pd, qd, pg, vset, tol=1e-13, max_iter=30)
    ok = r.status == CONVERGED or (r.status == MAX_ITER and r.final_mismatch < 1e-11)
    if not ok:
        raise RuntimeError(f"polished solve failed: status {r.status}, {r.final_mismatch}")
    return r.vm, r.va


def fd_gradient(Y, bus_type, pd, qd, pg, vset, which: str, coords, h=1e-6,
                loss_fn=loss):
    """Central differences (L(u + h e) - L(u - h e)) / 2h of ``loss_fn`` for
    the listed coordinates of input ``which`` in {pd, qd, pg, vset}."""
    base = {"pd": pd, "qd": qd, "pg": pg, "vset": vset}
    out = np.zeros(len(coords))
    for c, j in enumerate(coords):
        vals = []
        for s in (+1.0, -1.0):
            args = {k: v.copy() for k, v in base.items()}
            args[which][j] += s * h
            vm, va = solve_polished(Y, bus_type, args["pd"], args["qd"], args["pg"], args["vset"])
            vals.append(loss_fn(vm, va))
        out[c] = (vals[0] - vals[1]) / (2.0 * h)
    return out
