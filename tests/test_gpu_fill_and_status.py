"""GPU parity of the Jacobian value update as it lands in the LU positions,
and of the per-scenario stopping rule, against the CPU oracle.

The fill test reads the factor storage right after Algorithm 1's values are
written (``PF_EVAL_FILL``), before any elimination, in both residency modes
(LDS-resident slices of the 118-bus grid, HBM-resident slices of 16 scenarios
of the 1354-bus grid, and HBM-resident slices forced on the 118-bus grid),
rebuilds the dense J1 from the blocks and compares it with the oracle's
entry by entry; the PV padding entries and the fill-in blocks must be exact.
"""
import numpy as np
import pytest

from gpu_helpers import make_gpu_case, oracle_j1_paper, random_states, to_dev
from oracle.newton import Index, newton
from oracle.ybus import ybus_dense, ybus_of

pytestmark = pytest.mark.gpu


def _paper_positions(net):
    """Row of (dP_i, dQ_i) and column of (theta_j, |V|_j) of every bus in the
    paper's order (rows dP on B\\R then dQ on D; columns |V| on D then
    theta on B\\R), -1 where the unknown or equation does not exist."""
    idx = Index.of(net.bus_type)
    n = net.n_bus
    npvpq, npq = idx.pvpq.size, idx.pq.size
    rp, rq, ct, cv = (np.full(n, -1) for _ in range(4))
    rp[idx.pvpq] = np.arange(npvpq)
    rq[idx.pq] = npvpq + np.arange(npq)
    cv[idx.pq] = np.arange(npq)
    ct[idx.pvpq] = npq + np.arange(npvpq)
    return rp, rq, ct, cv


@pytest.mark.parametrize("name,precision,kw", [("c1", "fp64", {}), ("c1", "mixed", {}),
                                               ("c1", "mixed", {"block_threads": 256}),
                                               ("c2", "mixed", {}), ("c2", "fp64", {})])
def test_fill_writes_algorithm1_values_into_the_lu_positions(name, precision, kw, device):
    from paper_2606_07099_amd.pf import PF_EVAL_FILL
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, precision=precision, **kw)
    info = tpl.info()
    assert info["lds_resident"] == (0 if (name == "c2" or kw) else 1)
    count = 40 if name == "c2" else 12   # several slices and a ragged last one
    vm, va = random_states(net, count, 41)
    out = tpl.evaluate(PF_EVAL_FILL, d["pd"], d["qd"], d["pg"], d["vset"], to_dev(vm, device),
                       to_dev(va, device), count=count).cpu().numpy()
    rb, cb = tpl.block_pattern()
    nnzb = info["nnzb_lu"]
    assert out.shape == (count, 4 * nnzb)
    rp, rq, ct, cv = _paper_positions(net)
    bt = net.bus_type
    Y = ybus_of(net)
    in_y = np.abs(Y[rb, cb]) > 0            # blocks fed by a Y_bus entry; the others are fill-in
    # (Y entries that are present but exactly zero do not occur in these grids)
    nj = tpl.n_j
    for b in range(count):
        blk = out[b].reshape(nnzb, 2, 2)
        ref = oracle_j1_paper(net, vm[b], va[b])
        rebuilt = np.zeros((nj, nj))
        for p in range(nnzb):
            i, j = rb[p], cb[p]
            rows, cols = (rp[i], rq[i]), (ct[j], cv[j])
            for u in range(2):
                for w in range(2):
                    if rows[u] >= 0 and cols[w] >= 0:
                        rebuilt[rows[u], cols[w]] = blk[p, u, w]
                    else:   # padding of a PV bus: identity on its own |V| entry, else zero
                        assert blk[p, u, w] == (1.0 if (i == j and u == 1 and w == 1) else 0.0), (b, p, u, w)
            if not in_y[p]:
                assert not blk[p].any(), (b, p)
        scale = np.abs(ref).max()
        if precision == "fp64":
            assert np.abs(rebuilt - ref).max() <= 1e-13 * scale
        else:   # FP64 values rounded once to FP32
            assert np.all(np.abs(rebuilt - ref) <= 2.0 ** -24 * np.abs(ref) + 1e-14 * scale)
        assert np.array_equal(rebuilt != 0, ref != 0)
    assert bt[rb].size == nnzb


# ---------------------------------------------------------------- stopping rule

def _two_bus_template(precision, max_iter, batch=2):
    from paper_2606_07099_amd import PFTemplate
    R, X = 0.02, 0.1
    y = 1.0 / complex(R, X)
    indptr = np.array([0, 2, 4], np.int32)
    indices = np.array([0, 1, 0, 1], np.int32)
    g = np.array([y.real, -y.real, -y.real, y.real])
    b = np.array([y.imag, -y.imag, -y.imag, y.imag])
    bt = np.array([2, 0], np.int32)
    return PFTemplate(2, bt, indptr, indices, g, b, batch, tol=1e-8, max_iter=max_iter, precision=precision), bt


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("k", [1, 2])
def test_overload_status_and_iterations_match_oracle(precision, k, device):
    """Infeasible 2-bus load (no power-flow solution): status 1 after exactly
    max_iter updates on both sides; FP64 iterates equal the oracle's."""
    import torch
    tpl, bt = _two_bus_template(precision, k)
    P, Q = 5.0, 2.0
    pd = torch.tensor([[0.0, P], [0.0, 0.5]], dtype=torch.float64, device=device)
    qd = torch.tensor([[0.0, Q], [0.0, 0.2]], dtype=torch.float64, device=device)
    vset = torch.ones_like(pd)
    vm, va, iters, status, fn = (x.cpu().numpy() for x in tpl.solve(pd, qd, None, vset))
    Yd = ybus_dense(2, [0], [1], [0.02], [0.1], [0.0])
    for s in range(2):
        r = newton(Yd, bt, pd[s].cpu().numpy(), qd[s].cpu().numpy(), np.zeros(2), np.ones(2), tol=1e-8,
                   max_iter=k)
        assert int(status[s]) == r.status and int(iters[s]) == r.iters, (s, status[s], iters[s], r.status, r.iters)
        if precision == "fp64" or r.status == 0:
            assert abs(vm[s, 1] - r.vm[1]) <= 1e-8 and abs(va[s, 1] - r.va[1]) <= 1e-8
        if r.status == 1 and precision == "fp64":
            assert abs(fn[s] - r.final_mismatch) <= 1e-9 * max(1.0, r.final_mismatch)
    assert status[0] == 1 and iters[0] == k


def test_failure_statuses_match_oracle(device):
    """The 14-bus batch with one scenario loaded far beyond its limit and one
    with a NaN load: status and iteration count equal the oracle's on every
    scenario (max_iter 20: the overloaded scenario diverges without reaching
    non-finite values on either side)."""
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case("c0", device, batch=8)
    pd, qd = d["pd"].clone(), d["qd"].clone()
    pd[2] *= 8.0
    qd[2] *= 8.0
    pd[5, 3] = float("nan")
    vm, va, iters, status, fn = (x.cpu().numpy() for x in tpl.solve(pd, qd, d["pg"], d["vset"]))
    Y = ybus_of(net)
    pn, qn = pd.cpu().numpy(), qd.cpu().numpy()
    for b in range(8):
        r = newton(Y, net.bus_type, pn[b], qn[b], sc.pg[b], sc.vset[b], tol=tol)
        assert int(status[b]) == r.status and int(iters[b]) == r.iters, (b, status[b], iters[b], r.status, r.iters)
        if r.status == 2:
            assert np.isnan(fn[b])
        if r.status == 0:
            assert np.abs(vm[b] - r.vm).max() <= 1e-8
    assert status[2] == 1 and iters[2] == 20 and status[5] == 2 and iters[5] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_max_iter_zero_matches_oracle(precision, device):
    spec, net, sc, tpl, d, tol = make_gpu_case("c0", device, batch=4, max_iter=0, precision=precision)
    vm, va, iters, status, fn = (x.cpu().numpy() for x in tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"]))
    Y = ybus_of(net)
    for b in range(4):
        r = newton(Y, net.bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=tol, max_iter=0)
        assert int(status[b]) == r.status == 1 and int(iters[b]) == r.iters == 0
        assert abs(fn[b] - r.final_mismatch) <= 1e-12 * max(1.0, r.final_mismatch)
        assert np.array_equal(vm[b], r.vm) and np.array_equal(va[b], r.va)
