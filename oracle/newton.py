"""Step-1 Newton-Raphson completion, one scenario at a time (Sec. II-B).

For each scenario the unknowns are z1 = (V_m on PQ buses, theta on non-slack
buses) and the equations are F1 = (dP on non-slack buses, dQ on PQ buses) = 0
with dP = P_spec - P, dQ = Q_spec - Q, P_spec = p_g - p_d, Q_spec = q_g - q_d
(bus-type notation, Sec. II-A; reduced system and Newton step, Sec. II-B,
eqs. for F1, the linear system and J1).  PV and slack magnitudes are the
setpoints of the decision block x, the slack angle is 0, and the iteration
starts flat (|V| = 1 on PQ buses, angles 0; experimental setup, Sec. IV-A).

Readings where the paper is silent:

* convergence is ||F1||_inf < tol (strict), tested before every update,
  including at the flat start; ``iters`` counts the updates applied;
* a scenario with a non-finite mismatch stops with status 2; one still above
  tol after ``max_iter`` updates stops with status 1;
* generation is only read on PV buses; loads may sit on any non-slack bus
  (the synthetic grids put them on PQ buses only).

Unknown order here is (theta over non-slack buses ascending, then V_m over PQ
buses ascending) -- the paper's z1 lists V_m first; the order of the unknowns
does not change the Newton step.  The Jacobian is the derivative of the
calculated injection S = V * conj(Y V), formed with the complex-matrix forms

    dS/dtheta = j diag(V) conj(diag(I) - Y diag(V))
    dS/d|V|   = diag(V) conj(Y diag(V/|V|)) + conj(diag(I)) diag(V/|V|)

(a different route from the per-entry formulas of Algorithm 1, on purpose),
so J1 = dF1/dz1 = -[Re/Im of those rows and columns].  The linear system
J1 dz = -F1 is solved by LAPACK ``gesv`` with partial pivoting.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PQ, PV, SLACK = 0, 1, 2

CONVERGED, MAX_ITER, NON_FINITE = 0, 1, 2


@dataclass
class Index:
    """Bus partition of one network (Sec. II-A)."""
    pq: np.ndarray      # D, ascending
    pv: np.ndarray      # G, ascending
    ref: np.ndarray     # R (exactly one bus)
    pvpq: np.ndarray    # B \ R, ascending

    @staticmethod
    def of(bus_type) -> "Index":
        bt = np.asarray(bus_type)
        ref = np.flatnonzero(bt == SLACK)
        if ref.size != 1:
            raise ValueError("exactly one slack bus is required")
        return Index(np.flatnonzero(bt == PQ), np.flatnonzero(bt == PV), ref,
                     np.flatnonzero(bt != SLACK))


def calc_injection(Y: np.ndarray, V: np.ndarray) -> np.ndarray:
    """S = V * conj(Y V): calculated complex injection at every bus."""
    return V * np.conj(Y @ V)


def specified(pd, qd, pg, bus_type):
    """P_spec = p_g - p_d, Q_spec = q_g - q_d with generation read on PV buses only."""
    pv = np.asarray(bus_type) == PV
    p_spec = np.where(pv, pg, 0.0) - pd
    q_spec = -np.asarray(qd, dtype=np.float64)
    return p_spec, q_spec


def mismatch(Y, V, p_spec, q_spec, idx: Index) -> np.ndarray:
    """F1 = [P_spec - P]_(B\\R) || [Q_spec - Q]_D."""
    S = calc_injection(Y, V)
    return np.concatenate([p_spec[idx.pvpq] - S.real[idx.pvpq],
                           q_spec[idx.pq] - S.imag[idx.pq]])


def dS_dV(Y, V):
    """(dS/dtheta, dS/d|V|) as dense complex matrices over all buses."""
    # diag(a) @ M is written a[:, None] * M and M @ diag(a) is M * a[None, :]
    # (same products, without dense O(n^3) matmuls on the large grids).
    I = Y @ V
    Vn = V / np.abs(V)
    dVa = 1j * V[:, None] * np.conj(np.diag(I) - Y * V[None, :])
    dVm = V[:, None] * np.conj(Y * Vn[None, :]) + np.diag(np.conj(I) * Vn)
    return dVa, dVm


def jacobian_calc(Y, V, idx: Index) -> np.ndarray:
    """d(calc injection rows of F1)/d(theta_(B\\R), |V|_D) = -J1."""
    dVa, dVm = dS_dV(Y, V)
    r1, r2 = idx.pvpq, idx.pq
    return np.block([
        [dVa[np.ix_(r1, r1)].real, dVm[np.ix_(r1, r2)].real],
        [dVa[np.ix_(r2, r1)].imag, dVm[np.ix_(r2, r2)].imag],
    ])


def j1(Y, V, idx: Index) -> np.ndarray:
    """The paper's Step-1 Jacobian J1 = dF1/dz1 in this module's unknown order."""
    return -jacobian_calc(Y, V, idx)


@dataclass
class Result:
    vm: np.ndarray
    va: np.ndarray
    iters: int
    status: int
    final_mismatch: float
    history: list


def newton(Y, bus_type, pd, qd, pg, vset, tol=1e-8, max_iter=20,
           V0=None) -> Result:
    """Newton-Raphson from flat start for ONE scenario (all inputs per bus)."""
    idx = Index.of(bus_type)
    p_spec, q_spec = specified(pd, qd, pg, bus_type)
    n = len(bus_type)
    if V0 is None:
        vm = np.ones(n)
        vm[idx.pv] = vset[idx.pv]
        vm[idx.ref] = vset[idx.ref]
        va = np.zeros(n)
    else:
        vm, va = np.abs(V0).astype(np.float64), np.angle(V0).astype(np.float64)
    npvpq = idx.pvpq.size
    history = []
    t = 0
    while True:
        V = vm * np.exp(1j * va)
        F = mismatch(Y, V, p_spec, q_spec, idx)
        if not np.all(np.isfinite(F)):
            return Result(vm, va, t, NON_FINITE, float("nan"), history)
        nrm = float(np.max(np.abs(F))) if F.size else 0.0
        history.append(nrm)
        if nrm < tol:
            return Result(vm, va, t, CONVERGED, nrm, history)
        if t == max_iter:
            return Result(vm, va, t, MAX_ITER, nrm, history)
        J = j1(Y, V, idx)
        dz = np.linalg.solve(J, -F)
        va = va.copy()
        vm = vm.copy()
        va[idx.pvpq] += dz[:npvpq]
        vm[idx.pq] += dz[npvpq:]
        t += 1


@dataclass
class BatchResult:
    vm: np.ndarray       # [batch, n_bus]
    va: np.ndarray
    iters: np.ndarray    # int32 [batch]
    status: np.ndarray   # int32 [batch]
    final_mismatch: np.ndarray
    histories: list


def newton_batch(Y, bus_type, sc, tol=1e-8, max_iter=20, which=None) -> BatchResult:
    """Loop :func:`newton` over the scenarios of ``sc`` (each independent,
    as the block-diagonal embedding of Sec. III-A guarantees)."""
    which = range(sc.batch) if which is None else which
    out = [newton(Y, bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol, max_iter)
           for b in which]
    return BatchResult(np.stack([r.vm for r in out]), np.stack([r.va for r in out]),
                       np.array([r.iters for r in out], dtype=np.int32),
                       np.array([r.status for r in out], dtype=np.int32),
                       np.array([r.final_mismatch for r in out]),
                       [r.history for r in out])
