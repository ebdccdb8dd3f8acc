"""Pins of the oracle's Step-2 recovery and of the gradients of the full
two-step completion (Sec. II-B, eq. F2_completion, the chain-rule, J2 and
vbar2 equations).

Each compares the oracle with an independent route: branch-flow sums and
pi-model losses, the two-bus closed form (line losses R|I|^2 and X|I|^2 with
|I| = |S_load| / |V_2|, the load-bus voltage from its quartic), and central
differences of a loss on every completed output through polished solves.
"""
import numpy as np
import pytest

from gen.grids import make_case, PQ, PV, SLACK
from oracle.adjoint import adjoint, loss, loss_grad, solve_polished
from oracle.completion import (adjoint_completed, generation_loss, generation_loss_grad,
                               recover)
from oracle.newton import Index, newton, CONVERGED
from oracle.ybus import ybus_dense, ybus_of


def branch_flow_injection(n, f, t, r, x, bc, V):
    S = np.zeros(n, dtype=complex)
    for k in range(len(f)):
        a, b = f[k], t[k]
        ys = 1.0 / complex(r[k], x[k])
        S[a] += V[a] * np.conj(ys * (V[a] - V[b]) + 0.5j * bc[k] * V[a])
        S[b] += V[b] * np.conj(ys * (V[b] - V[a]) + 0.5j * bc[k] * V[b])
    return S


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_recovered_generation_matches_branch_flows_and_losses(name):
    spec, net, sc = make_case(name, batch=3)
    Y = ybus_of(net)
    bt = net.bus_type
    for b in range(3):
        r = newton(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=1e-11)
        assert r.status == CONVERGED
        pg_out, qg_out = recover(Y, bt, sc.pd[b], sc.qd[b], sc.pg[b], r.vm, r.va)
        V = r.vm * np.exp(1j * r.va)
        Sb = branch_flow_injection(net.n_bus, net.f, net.t, net.r, net.x, net.bc, V)
        gen = bt != PQ
        assert np.abs(qg_out[gen] - (Sb.imag[gen] + sc.qd[b][gen])).max() < 1e-10
        ref = bt == SLACK
        assert np.abs(pg_out[ref] - (Sb.real[ref] + sc.pd[b][ref])).max() < 1e-10
        assert np.all(pg_out[bt == PV] == sc.pg[b][bt == PV])
        assert np.all(pg_out[bt == PQ] == 0.0) and np.all(qg_out[bt == PQ] == 0.0)
        # system balance: generation - load = series I^2 r (active) and
        # I^2 x minus the charging of both line ends (reactive)
        p_loss = q_loss = 0.0
        for k in range(net.n_branch):
            a, c = net.f[k], net.t[k]
            i2 = abs((V[a] - V[c]) / complex(net.r[k], net.x[k])) ** 2
            p_loss += net.r[k] * i2
            q_loss += net.x[k] * i2 - 0.5 * net.bc[k] * (abs(V[a]) ** 2 + abs(V[c]) ** 2)
        assert abs(pg_out.sum() - sc.pd[b].sum() - p_loss) < 1e-9
        assert abs(qg_out.sum() - sc.qd[b].sum() - q_loss) < 1e-9


def two_bus_pq(P, Q, R, X):
    bt = np.array([SLACK, PQ], dtype=np.int32)
    Y = ybus_dense(2, [0], [1], [R], [X], [0.0])
    r = newton(Y, bt, np.array([0.0, P]), np.array([0.0, Q]), np.zeros(2), np.ones(2),
               tol=1e-13, max_iter=30)
    assert r.status == CONVERGED
    return bt, Y, r


@pytest.mark.parametrize("P,Q,R,X", [(0.5, 0.2, 0.02, 0.1), (0.9, 0.4, 0.03, 0.12)])
def test_recovery_and_its_gradient_two_bus_closed_form(P, Q, R, X):
    bt, Y, r = two_bus_pq(P, Q, R, X)
    w = r.vm[1] ** 2
    s2 = P * P + Q * Q
    pg_out, qg_out = recover(Y, bt, np.array([0.0, P]), np.array([0.0, Q]), np.zeros(2), r.vm, r.va)
    # the slack supplies the load plus the line losses, |I|^2 = |S|^2 / |V_2|^2
    assert abs(pg_out[0] - (P + R * s2 / w)) < 1e-11
    assert abs(qg_out[0] - (Q + X * s2 / w)) < 1e-11
    # d|V_2|^2 / dP and / dQ from differentiating the quartic in |V_2|^2
    a = P * R + Q * X
    c2 = R * R + X * X
    den = 2 * w + 2 * a - 1
    dw_dP = -(2 * R * w + 2 * P * c2) / den
    dw_dQ = -(2 * X * w + 2 * Q * c2) / den
    z = np.zeros(2)
    for coef, gp, gq in ((R, np.array([1.0, 0.0]), z), (X, z, np.array([1.0, 0.0]))):
        g = adjoint_completed(Y, bt, r.vm, r.va, z, z, gp, gq)
        want_p = (1.0 if coef == R else 0.0) + coef * (2 * P / w - s2 * dw_dP / w ** 2)
        want_q = (1.0 if coef == X else 0.0) + coef * (2 * Q / w - s2 * dw_dQ / w ** 2)
        assert abs(g.pd[1] - want_p) < 1e-10
        assert abs(g.qd[1] - want_q) < 1e-10
        # the slack's own load reaches its generation with unit weight
        assert g.pd[0] == gp[0] and g.qd[0] == gq[0]


def test_completed_adjoint_without_generation_terms_is_the_step1_adjoint():
    spec, net, sc = make_case("c0", batch=1)
    Y = ybus_of(net)
    r = newton(Y, net.bus_type, sc.pd[0], sc.qd[0], sc.pg[0], sc.vset[0], tol=1e-12)
    g_vm, g_va = loss_grad(r.vm, r.va)
    z = np.zeros(net.n_bus)
    a = adjoint_completed(Y, net.bus_type, r.vm, r.va, g_vm, g_va, z, z)
    b = adjoint(Y, net.bus_type, r.vm, r.va, g_vm, g_va)
    for k in ("pd", "qd", "pg", "vset"):
        assert np.allclose(getattr(a, k), getattr(b, k), rtol=1e-12, atol=1e-14)


def test_completed_adjoint_matches_central_differences_on_14_bus():
    spec, net, sc = make_case("c0", batch=2)
    Y = ybus_of(net)
    bt = net.bus_type
    idx = Index.of(bt)
    n = net.n_bus

    def total(pd, qd, pg, vset):
        vm, va = solve_polished(Y, bt, pd, qd, pg, vset)
        po, qo = recover(Y, bt, pd, qd, pg, vm, va)
        return loss(vm, va) + generation_loss(po, qo, bt)

    h = 1e-6
    for b in range(2):
        args = {"pd": sc.pd[b], "qd": sc.qd[b], "pg": sc.pg[b], "vset": sc.vset[b]}
        vm, va = solve_polished(Y, bt, *args.values())
        po, qo = recover(Y, bt, *(args[k] for k in ("pd", "qd", "pg")), vm, va)
        g_vm, g_va = loss_grad(vm, va)
        g_po, g_qo = generation_loss_grad(po, qo, bt)
        g = adjoint_completed(Y, bt, vm, va, g_vm, g_va, g_po, g_qo)
        for which, coords in (("pd", np.arange(n)), ("qd", np.arange(n)), ("pg", idx.pv),
                              ("vset", np.concatenate([idx.pv, idx.ref]))):
            fd = np.zeros(len(coords))
            for c, j in enumerate(coords):
                vals = []
                for s in (+1.0, -1.0):
                    a = {k: v.copy() for k, v in args.items()}
                    a[which][j] += s * h
                    vals.append(total(a["pd"], a["qd"], a["pg"], a["vset"]))
                fd[c] = (vals[0] - vals[1]) / (2 * h)
            an = getattr(g, which)[coords]
            assert np.linalg.norm(an - fd) <= 1e-6 * max(np.linalg.norm(fd), 1e-3), which
