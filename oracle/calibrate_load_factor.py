"""Choose the feasibility back-off ``load_factor`` of a synthetic grid.

Test infrastructure (calls only the oracle and the input generator).  The
synthetic recipe dispatches 0.95 of the total load on the PV buses and leaves
the rest plus all losses to the single slack bus; on the larger grids that
exceeds what the slack's few branches can carry and Newton diverges from the
flat start.  Reading adopted: scale every nominal load
(and therefore the dispatch) by 0.9**k with the smallest k for which the
nominal operating point converges from the flat start in at most 10 updates
with min |V| >= 0.90.  Feasibility is monotone in the load level over the
range probed, so k is found by bisection over k in [0, 64].

Usage:  python -m oracle.calibrate_load_factor c2
prints the factor to store in ``gen.grids.SPECS``.
"""
from __future__ import annotations

import dataclasses
import sys

import numpy as np

from gen.grids import SPECS, make_network
from oracle.newton import newton, CONVERGED
from oracle.ybus import ybus_of


def nominal_ok(name: str, factor: float, verbose=False) -> bool:
    spec = dataclasses.replace(SPECS[name], load_factor=1.0)
    net = make_network(spec)
    Y = ybus_of(net)
    pd, qd = net.p0 * factor, net.q0 * factor
    pg = np.zeros(net.n_bus)
    pg[net.pv] = 0.95 * pd.sum() / net.pv.size
    r = newton(Y, net.bus_type, pd, qd, pg, net.vset, tol=1e-8, max_iter=10)
    ok = r.status == CONVERGED and float(r.vm.min()) >= 0.90
    if verbose:
        print(f"  {name} factor={factor:.6g} status={r.status} iters={r.iters} "
              f"min|V|={r.vm.min():.4f} ok={ok}", flush=True)
    return ok


def calibrate(name: str, verbose=True) -> float:
    if nominal_ok(name, 1.0, verbose):
        return 1.0
    lo, hi = 0, 64
    if not nominal_ok(name, 0.9 ** hi, verbose):
        raise RuntimeError(f"{name}: no load factor down to 0.9**{hi} converges")
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if nominal_ok(name, 0.9 ** mid, verbose):
            hi = mid
        else:
            lo = mid
    return 0.9 ** hi


if __name__ == "__main__":
    for name in sys.argv[1:]:
        f = calibrate(name)
        print(f"{name}: load_factor = 0.9**{round(np.log(f) / np.log(0.9))} = {f!r}", flush=True)
