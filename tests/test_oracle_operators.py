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
