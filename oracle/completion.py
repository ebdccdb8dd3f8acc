"""Step-2 explicit recovery and the gradients of the whole two-step
completion, dense and one scenario at a time (Sec. II-B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward (eq. F2_completion): once z1 = (|V|_D, theta_(B\\R)) has converged,
the unused equality rows F2 = (dP on the slack bus, dQ on PV and slack buses)
are zero.  z2 = (p_g on the slack bus, q_g on PV and slack buses) enters F2
additively with unit coefficients, so z2 is the calculated injection plus the
load on those rows:

    p_g,R = P_R + p_d,R          q_g,i = Q_i + q_d,i   (i in B \\ D)

The completed generation block of y (eq. y_and_F_base) also holds p_g on PV
buses, which is the decision block x passed through.

Backward (chain-rule equation, J2 equation and the definitions that follow
it): with J2 = dF2/dv over the voltage block v = (|V|, theta) of every bus,

    vbar2 = -J2^T (dL/dz2)^T
    g_z1  = dL/dz1 + vbar2 restricted to z1
    g_x   = dL/dx  + vbar2 restricted to the |V| entries of x
    J1^T lambda = g_z1^T
    dL/dx = g_x - lambda^T dF1/dx,   dF1/dp_g,G = +I on the dP rows,
                                     dF1/d|V|_(B\\D) = J3.

The paper differentiates with respect to x only.  The loads u also reach the
outputs; this module returns those gradients too (reading listed with the
others): dF1/dp_d = -I on the dP rows gives lambda_P, and the direct unit
dependence of z2 on the load of its own row adds dL/dp_g,R to dL/dp_d at the
slack bus and dL/dq_g,i to dL/dq_d,i on PV and slack buses.  The slack angle
is fixed, so its entries of vbar2 are dropped.
"""
from __future__ import annotations

import numpy as np

from .adjoint import Grad
from .newton import Index, calc_injection, dS_dV, j1


def recover(Y, bus_type, pd, qd, pg, vm, va):
    """Completed generation (p_g, q_g) over all buses for ONE scenario: the
    Step-2 rows on slack (p_g) and PV + slack (q_g), x's p_g on PV buses,
    zero on PQ buses."""
    idx = Index.of(bus_type)
    S = calc_injection(Y, vm * np.exp(1j * va))
    n = len(bus_type)
    pg_out = np.zeros(n)
    qg_out = np.zeros(n)
    pg_out[idx.pv] = np.asarray(pg)[idx.pv]
    pg_out[idx.ref] = S.real[idx.ref] + np.asarray(pd)[idx.ref]
    gen = np.concatenate([idx.pv, idx.ref])
    qg_out[gen] = S.imag[gen] + np.asarray(qd)[gen]
    return pg_out, qg_out


def recover_batch(Y, bus_type, pd, qd, pg, vm, va):
    out = [recover(Y, bus_type, pd[b], qd[b], pg[b], vm[b], va[b]) for b in range(vm.shape[0])]
    return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


def j2(Y, V, idx: Index) -> np.ndarray:
    """J2 = dF2/dv, rows (dP_R, dQ_(B\\D)), columns (|V| of every bus, then
    theta of every bus); F = spec - calc, so J2 = -d(calc)/dv."""
    dVa, dVm = dS_dV(Y, V)
    gen = np.concatenate([idx.pv, idx.ref])
    return -np.block([
        [dVm[idx.ref, :].real, dVa[idx.ref, :].real],
        [dVm[gen, :].imag, dVa[gen, :].imag],
    ])


def j3(Y, V, idx: Index) -> np.ndarray:
    """J3 = dF1/d|V|_(B\\D): F1 rows (dP on B\\R, dQ on D), columns the PV
    then slack magnitudes."""
    _, dVm = dS_dV(Y, V)
    cols = np.concatenate([idx.pv, idx.ref])
    return -np.vstack([dVm[np.ix_(idx.pvpq, cols)].real, dVm[np.ix_(idx.pq, cols)].imag])


def adjoint_completed(Y, bus_type, vm, va, g_vm, g_va, g_pgo, g_qgo) -> Grad:
    """Gradients w.r.t. (p_d, q_d, p_g, V_set) for ONE converged scenario of
    a loss on every completed output: |V| and theta (g_vm, g_va) and the
    recovered generation (g_pgo on p_g, g_qgo on q_g, each over all buses;
    entries outside the rows that :func:`recover` fills are ignored)."""
    idx = Index.of(bus_type)
    n = len(bus_type)
    V = vm * np.exp(1j * va)
    gen = np.concatenate([idx.pv, idx.ref])
    # dL/dz2 in J2's row order, then vbar2 over (|V|, theta) of every bus
    g_z2 = np.concatenate([np.asarray(g_pgo)[idx.ref], np.asarray(g_qgo)[gen]])
    vbar2 = -j2(Y, V, idx).T @ g_z2
    vbar_vm, vbar_va = vbar2[:n], vbar2[n:]
    # accumulated row gradients (z1 in this package's order: theta, then |V|_D)
    g_z1 = np.concatenate([g_va[idx.pvpq] + vbar_va[idx.pvpq], g_vm[idx.pq] + vbar_vm[idx.pq]])
    g_x_vm = g_vm[gen] + vbar_vm[gen]
    g_x_pg = np.asarray(g_pgo)[idx.pv]            # p_g on PV buses is passed through
    lam = np.linalg.solve(j1(Y, V, idx).T, g_z1)
    npvpq = idx.pvpq.size
    lam_p = np.zeros(n)
    lam_q = np.zeros(n)
    lam_p[idx.pvpq] = lam[:npvpq]
    lam_q[idx.pq] = lam[npvpq:]
    g_pg = np.zeros(n)
    g_pg[idx.pv] = g_x_pg - lam_p[idx.pv]
    g_vset = np.zeros(n)
    g_vset[gen] = g_x_vm - j3(Y, V, idx).T @ lam
    g_pd = lam_p.copy()
    g_pd[idx.ref] += np.asarray(g_pgo)[idx.ref]
    g_qd = lam_q.copy()
    g_qd[gen] += np.asarray(g_qgo)[gen]
    return Grad(g_pd, g_qd, g_pg, g_vset, lam)


def adjoint_completed_batch(Y, bus_type, vm, va, g_vm, g_va, g_pgo, g_qgo) -> Grad:
    out = [adjoint_completed(Y, bus_type, vm[b], va[b], g_vm[b], g_va[b], g_pgo[b], g_qgo[b])
           for b in range(vm.shape[0])]
    return Grad(*(np.stack([getattr(o, k) for o in out]) for k in ("pd", "qd", "pg", "vset", "lam")))


def generation_loss(pg_out, qg_out, bus_type):
    """A loss on the recovered generation for tests and the benchmark:
    the sum over scenarios of p_g,R^2 + 0.5 * sum over PV and slack of q_g^2
    (a quadratic generation cost and a reactive-reserve penalty)."""
    bt = np.asarray(bus_type)
    slack = bt == 2
    gen = bt != 0
    return float(np.sum(pg_out[..., slack] ** 2) + 0.5 * np.sum(qg_out[..., gen] ** 2))


def generation_loss_grad(pg_out, qg_out, bus_type):
    bt = np.asarray(bus_type)
    g_p = np.where(bt == 2, 2.0 * pg_out, 0.0)
    g_q = np.where(bt != 0, qg_out, 0.0)
    return g_p, g_q

