"""The base Jacobian template and the operators the layer needs from it,
dense and one scenario at a time (Sec. II-A/II-B: eqs. y_and_F_base,
J_base_block, step1_jacobian, Jstep2_impl, Jstep3_impl; Sec. III-B,
block-aware indexing).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Orderings (the paper's, each block ascending by bus):

* y = (p_g on B\\D, q_g on B\\D, |V| of every bus, theta of every bus);
* F = (dP of every bus, dQ of every bus), dP = p_g - p_d - P, dQ = q_g - q_d - Q.

J = dF/dy: the generation columns are constant selectors (dP_i/dp_g,i = 1 and
dQ_i/dq_g,i = 1 on generator buses; the two cross blocks are zero) and the
voltage columns are -(dS/d|V|, dS/dtheta), real parts on the dP rows and
imaginary parts on the dQ rows.  The operators are sub-blocks of J:

* J1 = dF1/dz1: rows (dP on B\\R, dQ on D), columns z1 = (|V| on D, theta on B\\R);
* J2 = dF2/dv: rows (dP on R, dQ on B\\D), columns v = (|V|, theta) of every bus;
* J3 = dF1/d|V|_(B\\D): rows as J1, columns |V| on B\\D;

and the layer uses J1, J1^T, J2^T and J3^T.
"""
from __future__ import annotations

import numpy as np

from .newton import Index, dS_dV


def gen_buses(bus_type) -> np.ndarray:
    return np.flatnonzero(np.asarray(bus_type) != 0)


def base_jacobian(Y, bus_type, vm, va) -> np.ndarray:
    """Dense J = dF/dy, shape (2 n, 2 n_gen + 2 n)."""
    n = len(bus_type)
    gen = gen_buses(bus_type)
    ng = gen.size
    dVa, dVm = dS_dV(Y, vm * np.exp(1j * va))
    J = np.zeros((2 * n, 2 * ng + 2 * n))
    J[gen, np.arange(ng)] = 1.0                 # dP / dp_g selector
    J[n + gen, ng + np.arange(ng)] = 1.0        # dQ / dq_g selector
    J[:n, 2 * ng:2 * ng + n] = -dVm.real
    J[:n, 2 * ng + n:] = -dVa.real
    J[n:, 2 * ng:2 * ng + n] = -dVm.imag
    J[n:, 2 * ng + n:] = -dVa.imag
    return J


def operators(Y, bus_type, vm, va) -> dict:
    """{'J': J, 'J1': J1, 'J1T': J1^T, 'J2T': J2^T, 'J3T': J3^T} as dense
    sub-blocks of the base Jacobian."""
    idx = Index.of(bus_type)
    n = len(bus_type)
    gen = gen_buses(bus_type)
    ng = gen.size
    J = base_jacobian(Y, bus_type, vm, va)
    col_vm = 2 * ng
    col_va = 2 * ng + n
    f1_rows = np.concatenate([idx.pvpq, n + idx.pq])
    f2_rows = np.concatenate([idx.ref, n + gen])
    z1_cols = np.concatenate([col_vm + idx.pq, col_va + idx.pvpq])
    v_cols = np.arange(col_vm, 2 * ng + 2 * n)
    x_vm_cols = col_vm + gen
    J1 = J[np.ix_(f1_rows, z1_cols)]
    J2 = J[np.ix_(f2_rows, v_cols)]
    J3 = J[np.ix_(f1_rows, x_vm_cols)]
    return {"J": J, "J1": J1, "J1T": J1.T.copy(), "J2T": J2.T.copy(), "J3T": J3.T.copy()}
