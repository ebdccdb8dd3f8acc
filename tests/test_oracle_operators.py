"""Pins of the oracle's base Jacobian template and of the operators taken
from it: central differences of F(y) over every coordinate of y, the exact
selector blocks, and the structural pattern of Y_bus."""
import numpy as np
import pytest

from gen.grids import make_case
from oracle.newton import Index, calc_injection, j1
from oracle.operators import base_jacobian, gen_buses, operators
from oracle.ybus import ybus_of


def _F(Y, bt, pd, qd, y):
    n = len(bt)
    gen = gen_buses(bt)
    ng = gen.size
    pg = np.zeros(n)
    qg = np.zeros(n)
    pg[gen] = y[:ng]
    qg[gen] = y[ng:2 * ng]
    vm, va = y[2 * ng:2 * ng + n], y[2 * ng + n:]
    S = calc_injection(Y, vm * np.exp(1j * va))
    return np.concatenate([pg - pd - S.real, qg - qd - S.imag])


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_base_jacobian_matches_central_differences(name):
    spec, net, sc = make_case(name, batch=1)
    Y = ybus_of(net)
    bt = net.bus_type
    rng = np.random.default_rng(5)
    n = net.n_bus
    gen = gen_buses(bt)
    vm = rng.uniform(0.92, 1.08, n)
    va = rng.uniform(-0.3, 0.3, n)
    y = np.concatenate([rng.uniform(0, 1, gen.size), rng.uniform(-0.5, 0.5, gen.size), vm, va])
    J = base_jacobian(Y, bt, vm, va)
    h = 1e-6
    cols = range(J.shape[1]) if n < 50 else rng.choice(J.shape[1], 60, replace=False)
    for c in cols:
        e = np.zeros_like(y)
        e[c] = h
        fd = (_F(Y, bt, sc.pd[0], sc.qd[0], y + e) - _F(Y, bt, sc.pd[0], sc.qd[0], y - e)) / (2 * h)
        assert np.abs(fd - J[:, c]).max() <= 1e-6 * max(1.0, np.abs(J[:, c]).max()), c
    # the generation blocks are exact selectors, the cross blocks exact zeros
    ng = gen.size
    assert np.array_equal(J[:n, :ng], np.eye(n)[:, gen])
    assert np.array_equal(J[n:, ng:2 * ng], np.eye(n)[:, gen])
    assert not J[:n, ng:2 * ng].any() and not J[n:, :ng].any()


def test_operators_are_the_pinned_step1_jacobian_and_yield_its_transposes():
    spec, net, sc = make_case("c0", batch=1)
    Y = ybus_of(net)
    bt = net.bus_type
    rng = np.random.default_rng(8)
    vm = rng.uniform(0.92, 1.08, net.n_bus)
    va = rng.uniform(-0.3, 0.3, net.n_bus)
    ops = operators(Y, bt, vm, va)
    idx = Index.of(bt)
    # J1 of the Newton oracle has columns (theta_(B\R), |V|_D); the paper's are (|V|_D, theta_(B\R))
    ref = j1(Y, vm * np.exp(1j * va), idx)
    npvpq = idx.pvpq.size
    perm = np.concatenate([np.arange(npvpq, npvpq + idx.pq.size), np.arange(npvpq)])
    assert np.allclose(ops["J1"], ref[:, perm], rtol=0, atol=1e-13)
    assert np.array_equal(ops["J1T"], ops["J1"].T)
    n = net.n_bus
    ng = gen_buses(bt).size
    assert ops["J2T"].shape == (2 * n, 1 + ng)
    assert ops["J3T"].shape == (ng, idx.pvpq.size + idx.pq.size)


def test_voltage_blocks_follow_the_ybus_pattern():
    spec, net, sc = make_case("c0", batch=1)
    Y = ybus_of(net)
    bt = net.bus_type
    rng = np.random.default_rng(9)
    vm = rng.uniform(0.92, 1.08, net.n_bus)
    va = rng.uniform(-0.3, 0.3, net.n_bus)
    J = base_jacobian(Y, bt, vm, va)
    n = net.n_bus
    ng = gen_buses(bt).size
    pat = Y != 0
    for blk in (J[:n, 2 * ng:2 * ng + n], J[:n, 2 * ng + n:], J[n:, 2 * ng:2 * ng + n], J[n:, 2 * ng + n:]):
        assert np.all((blk != 0) <= pat)


# ---------------------------------------------------------------- J2 and J3 by differences
#
# The Step-2 rows F2 are the equality rows left out of F1 (eq. F2_completion):
# dP at the slack bus and dQ at every generator bus (B\D).  The mismatch here
# is formed from pi-model branch flows, not from Y_bus, so the pin shares no
# arithmetic with the oracle's operators; a wrong row block (dP for dQ), a
# wrong column block (theta for |V|) or a wrong sign fails it.

def _branch_flow_F(net, pd, qd, pg, qg, vm, va):
    """(dP, dQ) of every bus, with the calculated injection summed over the
    pi-model flows leaving each bus."""
    n = net.n_bus
    V = vm * np.exp(1j * va)
    S = np.zeros(n, dtype=complex)
    for k in range(net.n_branch):
        a, b = net.f[k], net.t[k]
        ys = 1.0 / complex(net.r[k], net.x[k])
        S[a] += V[a] * np.conj(ys * (V[a] - V[b]) + 0.5j * net.bc[k] * V[a])
        S[b] += V[b] * np.conj(ys * (V[b] - V[a]) + 0.5j * net.bc[k] * V[b])
    return pg - pd - S.real, qg - qd - S.imag


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_j2_and_j3_match_central_differences_of_the_left_out_rows(name):
    spec, net, sc = make_case(name, batch=1)
    bt = net.bus_type
    n = net.n_bus
    rng = np.random.default_rng(21)
    vm = rng.uniform(0.92, 1.08, n)
    va = rng.uniform(-0.3, 0.3, n)
    va[bt == 2] = 0.0
    pg = np.where(bt != 0, rng.uniform(0, 1, n), 0.0)
    qg = np.where(bt != 0, rng.uniform(-0.5, 0.5, n), 0.0)
    ops = operators(ybus_of(net), bt, vm, va)
    J2, J3 = ops["J2T"].T, ops["J3T"].T
    slack = np.flatnonzero(bt == 2)
    gen = np.flatnonzero(bt != 0)        # B \ D, ascending
    pvpq = np.flatnonzero(bt != 2)       # B \ R
    pq = np.flatnonzero(bt == 0)         # D

    def rows(vm_, va_):
        dP, dQ = _branch_flow_F(net, sc.pd[0], sc.qd[0], pg, qg, vm_, va_)
        return np.concatenate([dP[slack], dQ[gen]]), np.concatenate([dP[pvpq], dQ[pq]])

    assert J2.shape == (slack.size + gen.size, 2 * n)
    assert J3.shape == (pvpq.size + pq.size, gen.size)
    h = 1e-6
    cols = range(2 * n) if n < 50 else rng.choice(2 * n, 80, replace=False)
    for c in cols:   # v = (|V| of every bus, theta of every bus)
        dvm, dva = np.zeros(n), np.zeros(n)
        (dvm if c < n else dva)[c % n] = h
        f2p, _ = rows(vm + dvm, va + dva)
        f2m, _ = rows(vm - dvm, va - dva)
        fd = (f2p - f2m) / (2 * h)
        assert np.abs(fd - J2[:, c]).max() <= 1e-6 * max(1.0, np.abs(J2[:, c]).max()), c
    for k, i in enumerate(gen):          # |V| on B \ D
        dvm = np.zeros(n)
        dvm[i] = h
        fd = (rows(vm + dvm, va)[1] - rows(vm - dvm, va)[1]) / (2 * h)
        assert np.abs(fd - J3[:, k]).max() <= 1e-6 * max(1.0, np.abs(J3[:, k]).max()), i
    # the slack angle column of J2 is a real derivative too (the layer drops
    # it because the slack angle is fixed, not because it is zero)
    assert np.abs(J2[:, n + slack[0]]).max() > 0
