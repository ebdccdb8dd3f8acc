"""Dense bus admittance matrix Y_bus = G + jB (problem formulation, Sec. II-A).

The paper takes Y_bus from its test cases and states no branch model; the
synthetic grids use the standard pi model with series admittance
y_s = 1/(r + jx) and total line charging b split equally between the ends,
no tap ratios, phase shifters or bus shunts.
"""
from __future__ import annotations

import numpy as np


def ybus_dense(n_bus: int, f, t, r, x, bc) -> np.ndarray:
    """Complex [n_bus, n_bus] admittance matrix, one branch at a time."""
    Y = np.zeros((n_bus, n_bus), dtype=np.complex128)
    for k in range(len(f)):
        a, b = int(f[k]), int(t[k])
        ys = 1.0 / complex(r[k], x[k])
        ysh = 0.5j * bc[k]
        Y[a, a] += ys + ysh
        Y[b, b] += ys + ysh
        Y[a, b] -= ys
        Y[b, a] -= ys
    return Y


def ybus_of(net) -> np.ndarray:
    return ybus_dense(net.n_bus, net.f, net.t, net.r, net.x, net.bc)
