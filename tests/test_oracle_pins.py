"""Pins of the CPU oracle against what the physics and the paper fix.

None of these re-types the oracle's own formula: each compares it with an
independent route (branch-flow sums, polar textbook sums, finite differences,
closed-form two-bus solutions, the paper's printed Algorithm-1 entries,
invariants of S = V conj(Y V), brute-force root finding with scipy).
"""
import numpy as np
import pytest

from gen.grids import SPECS, make_case, PQ, PV, SLACK
from oracle.adjoint import adjoint, fd_gradient, loss, loss_grad
from oracle.newton import (Index, calc_injection, dS_dV, j1, mismatch, newton,
                           specified, CONVERGED)
from oracle.ybus import ybus_dense, ybus_of


def branch_flow_injection(n, f, t, r, x, bc, V):
    """Injection at each bus as the sum of pi-model branch flows leaving it."""
    S = np.zeros(n, dtype=complex)
    for k in range(len(f)):
        a, b = f[k], t[k]
        ys = 1.0 / complex(r[k], x[k])
        Iab = ys * (V[a] - V[b]) + 0.5j * bc[k] * V[a]
        Iba = ys * (V[b] - V[a]) + 0.5j * bc[k] * V[b]
        S[a] += V[a] * np.conj(Iab)
        S[b] += V[b] * np.conj(Iba)
    return S


def random_state(rng, n):
    vm = rng.uniform(0.9, 1.1, n)
    va = rng.uniform(-0.3, 0.3, n)
    return vm, va


# ---------------------------------------------------------------- Y_bus

def test_ybus_row_sums_without_charging():
    net = make_case("c1", batch=1)[1]
    Y = ybus_dense(net.n_bus, net.f, net.t, net.r, net.x, np.zeros_like(net.bc))
    assert np.abs(Y @ np.ones(net.n_bus)).max() < 1e-12
    assert np.abs(Y - Y.T).max() == 0.0


def test_ybus_row_sums_equal_half_charging():
    net = make_case("c1", batch=1)[1]
    Y = ybus_of(net)
    expect = np.zeros(net.n_bus, dtype=complex)
    for k in range(net.n_branch):
        expect[net.f[k]] += 0.5j * net.bc[k]
        expect[net.t[k]] += 0.5j * net.bc[k]
    assert np.abs(Y @ np.ones(net.n_bus) - expect).max() < 1e-12


def test_injection_equals_branch_flow_sum():
    net = make_case("c1", batch=1)[1]
    rng = np.random.default_rng(1)
    vm, va = random_state(rng, net.n_bus)
    V = vm * np.exp(1j * va)
    S1 = calc_injection(ybus_of(net), V)
    S2 = branch_flow_injection(net.n_bus, net.f, net.t, net.r, net.x, net.bc, V)
    assert np.abs(S1 - S2).max() < 1e-11


# ---------------------------------------------------------------- mismatch

def test_mismatch_at_flat_voltage_equals_spec():
    spec, net, sc = make_case("c0", batch=3)
    Y = ybus_dense(net.n_bus, net.f, net.t, net.r, net.x, np.zeros_like(net.bc))
    idx = Index.of(net.bus_type)
    for b in range(3):
        p, q = specified(sc.pd[b], sc.qd[b], sc.pg[b], net.bus_type)
        F = mismatch(Y, np.ones(net.n_bus, dtype=complex), p, q, idx)
        # Y @ 1 is zero up to the rounding of summing +y_s and -y_s
        np.testing.assert_allclose(F, np.concatenate([p[idx.pvpq], q[idx.pq]]), rtol=0, atol=1e-13)


def test_injection_matches_polar_textbook_sums():
    net = make_case("c0", batch=1)[1]
    Y = ybus_of(net)
    G, B = Y.real, Y.imag
    rng = np.random.default_rng(2)
    vm, va = random_state(rng, net.n_bus)
    S = calc_injection(Y, vm * np.exp(1j * va))
    n = net.n_bus
    P = np.zeros(n)
    Q = np.zeros(n)
    for i in range(n):
        for j in range(n):
            th = va[i] - va[j]
            P[i] += vm[i] * vm[j] * (G[i, j] * np.cos(th) + B[i, j] * np.sin(th))
            Q[i] += vm[i] * vm[j] * (G[i, j] * np.sin(th) - B[i, j] * np.cos(th))
    assert np.abs(S.real - P).max() < 1e-12
    assert np.abs(S.imag - Q).max() < 1e-12


# ---------------------------------------------------------------- Jacobian

def _f1_of_z(Y, bus_type, p, q, vm, va, z):
    idx = Index.of(bus_type)
    vm2, va2 = vm.copy(), va.copy()
    va2[idx.pvpq] = z[:idx.pvpq.size]
    vm2[idx.pq] = z[idx.pvpq.size:]
    return mismatch(Y, vm2 * np.exp(1j * va2), p, q, idx)


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_j1_matches_central_differences(name):
    spec, net, sc = make_case(name, batch=1)
    Y = ybus_of(net)
    idx = Index.of(net.bus_type)
    rng = np.random.default_rng(3)
    vm, va = random_state(rng, net.n_bus)
    p, q = specified(sc.pd[0], sc.qd[0], sc.pg[0], net.bus_type)
    z0 = np.concatenate([va[idx.pvpq], vm[idx.pq]])
    J = j1(Y, vm * np.exp(1j * va), idx)
    h = 1e-6
    Jfd = np.zeros_like(J)
    for c in range(z0.size):
        e = np.zeros_like(z0)
        e[c] = h
        Jfd[:, c] = (_f1_of_z(Y, net.bus_type, p, q, vm, va, z0 + e)
                     - _f1_of_z(Y, net.bus_type, p, q, vm, va, z0 - e)) / (2 * h)
    assert np.abs(J - Jfd).max() < 1e-6 * max(1.0, np.abs(J).max())


def test_dS_invariants_angle_shift_and_homogeneity():
    net = make_case("c1", batch=1)[1]
    Y = ybus_of(net)
    rng = np.random.default_rng(4)
    vm, va = random_state(rng, net.n_bus)
    V = vm * np.exp(1j * va)
    dVa, dVm = dS_dV(Y, V)
    S = calc_injection(Y, V)
    # rotating every angle together leaves S unchanged
    assert np.abs(dVa.sum(axis=1)).max() < 1e-10
    # S is homogeneous of degree 2 in the magnitudes (Euler)
    assert np.abs(dVm @ vm - 2.0 * S).max() < 1e-10


def _algorithm1_j1(Y, bus_type, vm, va):
    """J1 entries from the paper's Algorithm 1 (in-place value-update kernel):
    per (block, i, j) closed forms in V_m, V_re, V_im, I_re, I_im, theta."""
    idx = Index.of(bus_type)
    V = vm * np.exp(1j * va)
    I = Y @ V
    vre, vim, ire, iim = V.real, V.imag, I.real, I.imag
    G, B = Y.real, Y.imag

    def eta(blk, i, j):
        g, b = G[i, j], B[i, j]
        th = va[i] - va[j]
        if blk == "dP_theta":
            if i == j:
                return vim[i] * ire[i] - vre[i] * iim[i] + b * vm[i] ** 2
            return -vm[i] * vm[j] * (g * np.sin(th) - b * np.cos(th))
        if blk == "dP_vm":
            if i == j:
                return -(vre[i] * ire[i] + vim[i] * iim[i]) / vm[i] - g * vm[i]
            return -vm[i] * (g * np.cos(th) + b * np.sin(th))
        if blk == "dQ_theta":
            if i == j:
                return -(vre[i] * ire[i] + vim[i] * iim[i]) + g * vm[i] ** 2
            return vm[i] * vm[j] * (g * np.cos(th) + b * np.sin(th))
        if blk == "dQ_vm":
            if i == j:
                return -(vim[i] * ire[i] - vre[i] * iim[i]) / vm[i] + b * vm[i]
            return -vm[i] * (g * np.sin(th) - b * np.cos(th))
        raise KeyError(blk)

    rows = [("P", i) for i in idx.pvpq] + [("Q", i) for i in idx.pq]
    cols = [("theta", j) for j in idx.pvpq] + [("vm", j) for j in idx.pq]
    J = np.zeros((len(rows), len(cols)))
    for r, (rk, i) in enumerate(rows):
        for c, (ck, j) in enumerate(cols):
            J[r, c] = eta(f"d{rk}_{ck}", i, j)
    return J


def test_j1_matches_paper_algorithm1_entries():
    spec, net, sc = make_case("c0", batch=1)
    Y = ybus_of(net)
    rng = np.random.default_rng(5)
    vm, va = random_state(rng, net.n_bus)
    J_or = j1(Y, vm * np.exp(1j * va), Index.of(net.bus_type))
    J_alg = _algorithm1_j1(Y, net.bus_type, vm, va)
    assert np.abs(J_or - J_alg).max() < 1e-12 * max(1.0, np.abs(J_or).max())


# ---------------------------------------------------------------- two-bus closed forms

def two_bus(R, X, bus2_type):
    bt = np.array([SLACK, bus2_type], dtype=np.int32)
    Y = ybus_dense(2, [0], [1], [R], [X], [0.0])
    return bt, Y


@pytest.mark.parametrize("P,Q,R,X", [(0.5, 0.2, 0.02, 0.1), (1.0, 0.3, 0.01, 0.08),
                                     (0.3, -0.1, 0.05, 0.2), (0.0, 0.0, 0.03, 0.1)])
def test_two_bus_slack_pq_closed_form(P, Q, R, X):
    bt, Y = two_bus(R, X, PQ)
    r = newton(Y, bt, np.array([0.0, P]), np.array([0.0, Q]), np.zeros(2),
               np.array([1.0, 1.0]), tol=1e-12, max_iter=30)
    assert r.status == CONVERGED
    a = P * R + Q * X
    c = (P * P + Q * Q) * (R * R + X * X)
    w = ((1 - 2 * a) + np.sqrt((1 - 2 * a) ** 2 - 4 * c)) / 2
    U = np.sqrt(w)
    delta = np.arctan2(Q * R - P * X, w + a)
    assert abs(r.vm[1] - U) < 1e-11
    assert abs(r.va[1] - delta) < 1e-11
    assert r.vm[0] == 1.0 and r.va[0] == 0.0


@pytest.mark.parametrize("P2,U,R,X", [(0.4, 1.02, 0.02, 0.1), (-0.6, 0.99, 0.01, 0.05)])
def test_two_bus_slack_pv_closed_form(P2, U, R, X):
    bt, Y = two_bus(R, X, PV)
    r = newton(Y, bt, np.zeros(2), np.zeros(2), np.array([0.0, P2]),
               np.array([1.0, U]), tol=1e-12, max_iter=30)
    assert r.status == CONVERGED
    G22, G21, B21 = Y[1, 1].real, Y[1, 0].real, Y[1, 0].imag
    c = (P2 - G22 * U * U) / U
    M = np.hypot(G21, B21)
    phi = np.arctan2(B21, G21)
    roots = [phi + s * np.arccos(c / M) for s in (+1, -1)]
    roots = [np.angle(np.exp(1j * d)) for d in roots]
    delta = min(roots, key=abs)
    assert abs(r.va[1] - delta) < 1e-11
    assert r.vm[1] == U


# ---------------------------------------------------------------- Newton behaviour

def test_zero_injection_flat_solution_needs_no_update():
    net = make_case("c0", batch=1)[1]
    Y = ybus_dense(net.n_bus, net.f, net.t, net.r, net.x, np.zeros_like(net.bc))
    n = net.n_bus
    r = newton(Y, net.bus_type, np.zeros(n), np.zeros(n), np.zeros(n), np.ones(n))
    assert r.status == CONVERGED and r.iters == 0
    assert np.all(r.vm == 1.0) and np.all(r.va == 0.0)


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_power_balance_at_convergence(name):
    spec, net, sc = make_case(name, batch=4)
    Y = ybus_of(net)
    for b in range(4):
        r = newton(Y, net.bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=1e-10)
        assert r.status == CONVERGED and r.final_mismatch < 1e-10
        V = r.vm * np.exp(1j * r.va)
        S = calc_injection(Y, V)
        losses = 0.0
        for k in range(net.n_branch):
            ys = 1.0 / complex(net.r[k], net.x[k])
            losses += net.r[k] * abs(ys * (V[net.f[k]] - V[net.t[k]])) ** 2
        assert abs(S.real.sum() - losses) < 1e-9
        # the specified injections hold on every F1 row
        idx = Index.of(net.bus_type)
        p, q = specified(sc.pd[b], sc.qd[b], sc.pg[b], net.bus_type)
        assert np.abs(S.real[idx.pvpq] - p[idx.pvpq]).max() < 1e-10
        assert np.abs(S.imag[idx.pq] - q[idx.pq]).max() < 1e-10


def test_quadratic_convergence():
    spec, net, sc = make_case("c1", batch=1)
    r = newton(ybus_of(net), net.bus_type, sc.pd[0], sc.qd[0], sc.pg[0], sc.vset[0], tol=1e-12)
    h = r.history
    assert r.status == CONVERGED and len(h) >= 4
    # ||F_{t+1}|| <= C ||F_t||^2 once in the quadratic regime
    for t in range(1, len(h) - 1):
        if h[t] < 1e-2 and h[t + 1] > 1e-13:
            assert h[t + 1] <= 50.0 * h[t] ** 2


def test_relabelling_buses_permutes_the_solution():
    spec, net, sc = make_case("c0", batch=2)
    rng = np.random.default_rng(6)
    perm = rng.permutation(net.n_bus)           # new bus k is old bus perm[k]
    inv = np.argsort(perm)
    Y = ybus_of(net)
    Yp = ybus_dense(net.n_bus, inv[net.f], inv[net.t], net.r, net.x, net.bc)
    for b in range(2):
        r0 = newton(Y, net.bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b])
        r1 = newton(Yp, net.bus_type[perm], sc.pd[b][perm], sc.qd[b][perm], sc.pg[b][perm],
                    sc.vset[b][perm])
        assert r0.iters == r1.iters
        assert np.abs(r1.vm - r0.vm[perm]).max() < 1e-12
        assert np.abs(r1.va - r0.va[perm]).max() < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_newton_root_is_the_high_voltage_root_among_brute_force_roots(seed):
    """3- and 4-bus meshes: multistart scipy root finding on a branch-flow
    residual finds every root it can; the oracle's root is one of them and
    is the one with the highest PQ-bus voltages (the normal operating point)."""
    from scipy.optimize import root
    rng = np.random.default_rng(100 + seed)
    n = 3 + seed
    f = [0, 1, 0] + ([2] if n == 4 else [])
    t = [1, 2, 2] + ([3] if n == 4 else [])
    m = len(f)
    r_ = rng.uniform(0.01, 0.05, m)
    x_ = r_ * rng.uniform(3, 10, m)
    bc = rng.uniform(0, 0.05, m)
    bt = np.array([SLACK, PQ, PV] + ([PQ] if n == 4 else []), dtype=np.int32)
    pd = np.array([0, 0.8, 0] + ([0.5] if n == 4 else []))
    qd = 0.3 * pd
    pg = np.array([0, 0, 0.6] + ([0] if n == 4 else []))
    vset = np.array([1.0, 1.0, 1.02] + ([1.0] if n == 4 else []))
    Y = ybus_dense(n, f, t, r_, x_, bc)
    idx = Index.of(bt)
    pspec = np.where(bt == PV, pg, 0) - pd
    qspec = -qd

    def resid(z):
        va = np.zeros(n)
        vm = vset.copy()
        va[idx.pvpq] = z[:idx.pvpq.size]
        vm[idx.pq] = z[idx.pvpq.size:]
        S = branch_flow_injection(n, f, t, r_, x_, bc, vm * np.exp(1j * va))
        return np.concatenate([pspec[idx.pvpq] - S.real[idx.pvpq], qspec[idx.pq] - S.imag[idx.pq]])

    roots = []
    grid_a = np.linspace(-1.2, 1.2, 5)
    grid_v = [0.2, 0.5, 0.8, 1.0, 1.2]
    import itertools
    for za in itertools.product(grid_a, repeat=idx.pvpq.size):
        for zv in itertools.product(grid_v, repeat=idx.pq.size):
            s = root(resid, np.array(za + zv), method="hybr", tol=1e-13)
            if s.success and np.abs(resid(s.x)).max() < 1e-9:
                z = s.x.copy()
                z[:idx.pvpq.size] = np.angle(np.exp(1j * z[:idx.pvpq.size]))
                if not any(np.abs(z - q).max() < 1e-6 for q in roots):
                    roots.append(z)
    r = newton(Y, bt, pd, qd, pg, vset, tol=1e-12)
    assert r.status == CONVERGED
    z_or = np.concatenate([r.va[idx.pvpq], r.vm[idx.pq]])
    d = [np.abs(z_or - q).max() for q in roots]
    assert min(d) < 1e-8
    hv = max(roots, key=lambda q: q[idx.pvpq.size:].min())
    assert np.abs(z_or - hv).max() < 1e-8


# ---------------------------------------------------------------- adjoint

def test_loss_gradient_matches_differences():
    rng = np.random.default_rng(7)
    vm = rng.uniform(0.9, 1.1, 40)
    va = rng.uniform(-0.5, 0.5, 40)
    g_vm, g_va = loss_grad(vm, va)
    h = 1e-7
    for i in range(40):
        e = np.zeros(40)
        e[i] = h
        assert abs((loss(vm + e, va) - loss(vm - e, va)) / (2 * h) - g_vm[i]) < 1e-6
        assert abs((loss(vm, va + e) - loss(vm, va - e)) / (2 * h) - g_va[i]) < 1e-6


@pytest.mark.parametrize("P,Q,R,X", [(0.5, 0.2, 0.02, 0.1), (0.9, 0.4, 0.03, 0.12)])
def test_adjoint_two_bus_slack_pq_closed_form(P, Q, R, X):
    bt, Y = two_bus(R, X, PQ)
    r = newton(Y, bt, np.array([0.0, P]), np.array([0.0, Q]), np.zeros(2), np.ones(2), tol=1e-13,
               max_iter=30)
    # L = |V_2| + theta_2: dL/dp_d and dL/dq_d from differentiating the quartic
    a = P * R + Q * X
    c2 = R * R + X * X
    w = r.vm[1] ** 2
    U = r.vm[1]
    den = 2 * w + 2 * a - 1
    dw_dP = -(2 * R * w + 2 * P * c2) / den
    dw_dQ = -(2 * X * w + 2 * Q * c2) / den
    s = Q * R - P * X
    cc = w + a

    def ddelta(ds, dcc):
        return (cc * ds - s * dcc) / (cc * cc + s * s)

    dL_dP = dw_dP / (2 * U) + ddelta(-X, dw_dP + R)
    dL_dQ = dw_dQ / (2 * U) + ddelta(R, dw_dQ + X)
    g = adjoint(Y, bt, r.vm, r.va, np.array([0.0, 1.0]), np.array([0.0, 1.0]))
    assert abs(g.pd[1] - dL_dP) < 1e-10
    assert abs(g.qd[1] - dL_dQ) < 1e-10


def test_adjoint_two_bus_slack_pv_closed_form():
    bt, Y = two_bus(0.02, 0.1, PV)
    U, P2 = 1.02, 0.4
    r = newton(Y, bt, np.zeros(2), np.zeros(2), np.array([0.0, P2]), np.array([1.0, U]), tol=1e-13,
               max_iter=30)
    G22, G21, B21 = Y[1, 1].real, Y[1, 0].real, Y[1, 0].imag
    d = r.va[1]
    dP_ddelta = U * (-G21 * np.sin(d) + B21 * np.cos(d))
    dP_dU = 2 * G22 * U + (G21 * np.cos(d) + B21 * np.sin(d))
    # L = theta_2 + 3 |V_2|: theta_2 moves with p_g and with the setpoint
    g = adjoint(Y, bt, r.vm, r.va, np.array([0.0, 3.0]), np.array([0.0, 1.0]))
    assert abs(g.pg[1] - 1.0 / dP_ddelta) < 1e-10
    assert abs(g.vset[1] - (3.0 - dP_dU / dP_ddelta)) < 1e-10


def test_adjoint_matches_central_differences_on_14_bus():
    spec, net, sc = make_case("c0", batch=2)
    Y = ybus_of(net)
    for b in range(2):
        r = newton(Y, net.bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=1e-13, max_iter=30)
        g_vm, g_va = loss_grad(r.vm, r.va)
        g = adjoint(Y, net.bus_type, r.vm, r.va, g_vm, g_va)
        idx = Index.of(net.bus_type)
        for which, coords in (("pd", idx.pvpq), ("qd", idx.pq), ("pg", idx.pv),
                              ("vset", np.concatenate([idx.pv, idx.ref]))):
            fd = fd_gradient(Y, net.bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], which, coords)
            an = getattr(g, which)[coords]
            assert np.linalg.norm(an - fd) <= 1e-6 * max(np.linalg.norm(fd), 1e-3), which


# ---------------------------------------------------------------- statuses
#
# Readings of the stopping rule (the paper gives only the tolerance): the
# test ||F1||_inf < tol runs before every update, iters counts the updates
# applied, a scenario still at or above tol after max_iter updates stops
# with status 1, and a non-finite mismatch stops it with status 2.

def _two_bus_pq_step(P, Q, R, X, U, d):
    """One Newton update of the 2-bus slack-PQ network from (|V2|, theta2),
    with F = spec - calc formed from the branch flow V2 conj((V2 - 1)/z)
    and a central-difference Jacobian (independent of the oracle's)."""
    z = complex(R, X)

    def F(u):
        V2 = u[1] * np.exp(1j * u[0])
        S2 = V2 * np.conj((V2 - 1.0) / z)
        return np.array([-P - S2.real, -Q - S2.imag])

    u = np.array([d, U])
    h = 1e-7
    J = np.column_stack([(F(u + h * e) - F(u - h * e)) / (2 * h) for e in np.eye(2)])
    du = np.linalg.solve(J, -F(u))
    return u[1] + du[1], u[0] + du[0]


@pytest.mark.parametrize("k", [1, 2])
def test_overload_stops_after_exactly_max_iter_updates(k):
    """Load beyond the 2-bus loadability limit (negative discriminant of the
    quartic in |V2|^2, so no power-flow solution exists): Newton cannot
    converge, and with max_iter = k the oracle returns status 1 after exactly
    k updates, the k-th one being a Newton step from the state after k - 1.
    (k <= 2: the third step would start from a negative |V2|, outside the
    domain where the oracle's derivative forms, which divide by |V|, are
    those of the magnitude variable.)"""
    P, Q, R, X = 5.0, 2.0, 0.02, 0.1
    a = P * R + Q * X
    assert (1 - 2 * a) ** 2 - 4 * (P * P + Q * Q) * (R * R + X * X) < 0
    bt, Y = two_bus(R, X, PQ)
    args = (Y, bt, np.array([0.0, P]), np.array([0.0, Q]), np.zeros(2), np.ones(2))
    r = newton(*args, tol=1e-8, max_iter=k)
    prev = newton(*args, tol=1e-8, max_iter=k - 1)
    assert r.status == 1 and r.iters == k and len(r.history) == k + 1
    assert prev.status == 1 and prev.iters == k - 1
    U, d = _two_bus_pq_step(P, Q, R, X, prev.vm[1], prev.va[1])
    assert abs(r.vm[1] - U) < 1e-6 * max(1.0, abs(U)) and abs(r.va[1] - d) < 1e-6 * max(1.0, abs(d))
    # the reported mismatch is the one at the returned state
    S2 = r.vm[1] * np.exp(1j * r.va[1]) * np.conj((r.vm[1] * np.exp(1j * r.va[1]) - 1.0) / complex(R, X))
    assert abs(r.final_mismatch - max(abs(-P - S2.real), abs(-Q - S2.imag))) < 1e-9 * max(1.0, r.final_mismatch)


def test_max_iter_zero_only_evaluates_the_flat_start():
    """max_iter = 0: no update, status 1 for a loaded network, and the
    reported mismatch is the flat-start one, which without line charging is
    the specified injection itself (the calculated injection is 0)."""
    spec, net, sc = make_case("c0", batch=1)
    Y = ybus_dense(net.n_bus, net.f, net.t, net.r, net.x, np.zeros_like(net.bc))
    vset = np.ones(net.n_bus)
    r = newton(Y, net.bus_type, sc.pd[0], sc.qd[0], sc.pg[0], vset, max_iter=0)
    assert r.status == 1 and r.iters == 0
    p, q = specified(sc.pd[0], sc.qd[0], sc.pg[0], net.bus_type)
    idx = Index.of(net.bus_type)
    expect = max(np.abs(p[idx.pvpq]).max(), np.abs(q[idx.pq]).max())
    assert abs(r.final_mismatch - expect) < 1e-13
    assert np.all(r.vm == vset) and np.all(r.va == 0.0)


@pytest.mark.parametrize("where", ["pd", "qd", "pg"])
def test_non_finite_input_stops_at_the_flat_start_with_status_2(where):
    spec, net, sc = make_case("c0", batch=1)
    Y = ybus_of(net)
    x = {k: getattr(sc, k)[0].copy() for k in ("pd", "qd", "pg", "vset")}
    bus = int(np.flatnonzero(net.bus_type == (PV if where == "pg" else PQ))[0])
    x[where][bus] = np.nan
    r = newton(Y, net.bus_type, x["pd"], x["qd"], x["pg"], x["vset"])
    assert r.status == 2 and r.iters == 0 and np.isnan(r.final_mismatch)
    # generation on a PQ bus is not read (it is zero by definition), so a NaN
    # there changes nothing
    x = {k: getattr(sc, k)[0].copy() for k in ("pd", "qd", "pg", "vset")}
    x["pg"][int(np.flatnonzero(net.bus_type == PQ)[0])] = np.nan
    r = newton(Y, net.bus_type, x["pd"], x["qd"], x["pg"], x["vset"])
    assert r.status == CONVERGED
