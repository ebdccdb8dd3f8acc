"""The C ABI from a plain C program (paper_2606_07099_amd/csrc/abi_check.c,
built next to the library): no Python or torch in the process.  It builds a
template from a branch list, solves a batch and runs the adjoint of
L = sum |V| + sum theta; the results must match the oracle."""
import os
import subprocess

import numpy as np
import pytest

from gen.grids import make_case
from oracle.adjoint import adjoint
from oracle.newton import newton
from oracle.ybus import ybus_of

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2606_07099_amd", "abi_check")


@pytest.mark.parametrize("precision", [0, 1])
def test_plain_c_client_matches_oracle(precision, tmp_path, device):
    if not os.path.exists(EXE):
        raise FileNotFoundError(f"{EXE} is not built (python -m paper_2606_07099_amd.build)")
    spec, net, sc = make_case("c0", batch=6)
    n, m, B = net.n_bus, net.n_branch, sc.batch
    lines = [f"{n} {m} {B} {precision}", " ".join(map(str, net.bus_type)),
             " ".join(map(str, net.f)), " ".join(map(str, net.t))]
    lines += [" ".join(repr(float(v)) for v in arr) for arr in (net.r, net.x, net.bc)]
    lines += [" ".join(repr(float(v)) for v in getattr(sc, k).ravel()) for k in ("pd", "qd", "pg", "vset")]
    inp = tmp_path / "case.txt"
    inp.write_text("\n".join(lines) + "\n")
    print(f"abi_check precision={precision}", flush=True)
    r = subprocess.run([EXE, str(inp)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rows = [np.array(l.split(), dtype=float) for l in r.stdout.strip().splitlines()]
    assert len(rows) == B
    Y = ybus_of(net)
    for b, row in enumerate(rows):
        status, iters = int(row[0]), int(row[1])
        vm, va, gpd, gqd, gpg, gvs = row[2:].reshape(6, n)
        ref = newton(Y, net.bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=1e-10)
        assert status == 0
        assert iters - ref.iters in ((0,) if precision == 0 else (0, 1))
        assert np.abs(vm - ref.vm).max() <= 1e-8 and np.abs(va - ref.va).max() <= 1e-8
        g = adjoint(Y, net.bus_type, ref.vm, ref.va, np.ones(n), np.ones(n))
        ours = np.concatenate([gpd, gqd, gpg, gvs])
        want = np.concatenate([g.pd, g.qd, g.pg, g.vset])
        assert np.linalg.norm(ours - want) <= 1e-6 * np.linalg.norm(want)
