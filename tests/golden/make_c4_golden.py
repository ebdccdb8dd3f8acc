"""Writes ``c4_subset.npz``: the CPU oracle's results for three fixed
scenarios of the 9241-bus batch of 256 (seed 0, lognormal load scenarios,
tolerance 1e-8), for the GPU parity test of that grid.

Calls only ``gen`` (the seeded inputs) and ``oracle`` (dense FP64 Newton with
LAPACK and the dense adjoint): the Step-1 Newton completion from the flat
start (Sec. II-B; flat start and tolerance of Sec. IV-A) and the
implicit-differentiation gradients of the layer loss at its solution
(backward pass of Sec. II-B).  The dense Jacobian has 17k x 17k entries, so
each scenario takes a few minutes and about 15 GB of memory.

    python tests/golden/make_c4_golden.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from gen.grids import SPECS, make_case  # noqa: E402
from oracle.adjoint import adjoint, loss_grad  # noqa: E402
from oracle.newton import newton  # noqa: E402
from oracle.ybus import ybus_of  # noqa: E402

SCENARIOS = (0, 97, 255)
OUT = os.path.join(HERE, "c4_subset.npz")


def main():
    spec, net, sc = make_case("c4")
    assert sc.batch == SPECS["c4"].batch == 256
    Y = ybus_of(net)
    res = {k: [] for k in ("vm", "va", "iters", "status", "final_mismatch", "g_pd", "g_qd", "g_pg", "g_vset")}
    hist = []
    for b in SCENARIOS:
        t0 = time.time()
        r = newton(Y, net.bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=spec.tol)
        assert r.status == 0, (b, r.status)
        g_vm, g_va = loss_grad(r.vm, r.va)
        g = adjoint(Y, net.bus_type, r.vm, r.va, g_vm, g_va)
        for k, v in (("vm", r.vm), ("va", r.va), ("iters", r.iters), ("status", r.status),
                     ("final_mismatch", r.final_mismatch), ("g_pd", g.pd), ("g_qd", g.qd), ("g_pg", g.pg),
                     ("g_vset", g.vset)):
            res[k].append(v)
        hist.append(np.pad(np.asarray(r.history), (0, 32 - len(r.history)), constant_values=np.nan))
        print(f"scenario {b}: {r.iters} updates, final {r.final_mismatch:.3e}, {time.time() - t0:.0f} s",
              flush=True)
    np.savez_compressed(OUT, scenarios=np.array(SCENARIOS, np.int32), seed=np.int32(0),
                        grid=np.array("c4"), batch=np.int32(sc.batch), tol=np.float64(spec.tol),
                        history=np.stack(hist), **{k: np.array(v) for k, v in res.items()})
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
