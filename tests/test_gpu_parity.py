"""GPU parity of the HIP path against the CPU FP64 oracle, through the C ABI.

Kernel level (mismatch, Jacobian fill, Newton step, adjoint solve) at random
states, end to end (Newton from the flat start) on every grid in the launch
configuration of the benchmark, sampled where the dense oracle is slow.
Tolerances: |V| within 1e-8 pu and angles within 1e-8 rad, identical
iteration counts and statuses in FP64; the mixed-precision path within the
same voltage bounds and at most one extra iteration.
"""
import numpy as np
import pytest

from gpu_helpers import (make_gpu_case, oracle_f1, oracle_j1_paper, paper_col_perm,
                         random_states, tie_band, to_dev)
from oracle.newton import newton_batch, newton
from oracle.ybus import ybus_of

pytestmark = pytest.mark.gpu


def _states(net, device, count, seed):
    vm, va = random_states(net, count, seed)
    return vm, va, to_dev(vm, device), to_dev(va, device)


# ---------------------------------------------------------------- kernel level

@pytest.mark.parametrize("name", ["c0", "c1", "c3"])
def test_mismatch_kernel_matches_oracle(name, device):
    from paper_2606_07099_amd.pf import PF_EVAL_MISMATCH
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device)
    count = min(sc.batch, 8)
    vm, va, tvm, tva = _states(net, device, count, 11)
    out = tpl.evaluate(PF_EVAL_MISMATCH, d["pd"], d["qd"], d["pg"], d["vset"], tvm, tva,
                       count=count).cpu().numpy()
    for b in range(count):
        ref = oracle_f1(net, sc, b, vm[b], va[b])
        assert np.abs(out[b] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("name", ["c0", "c1", "c3"])
def test_jacobian_fill_matches_oracle(name, device):
    from paper_2606_07099_amd.pf import PF_EVAL_JACOBIAN
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device)
    count = min(sc.batch, 4)
    vm, va, tvm, tva = _states(net, device, count, 12)
    out = tpl.evaluate(PF_EVAL_JACOBIAN, d["pd"], d["qd"], d["pg"], d["vset"], tvm, tva,
                       count=count).cpu().numpy()
    for b in range(count):
        ref = oracle_j1_paper(net, vm[b], va[b])
        assert np.array_equal(out[b] != 0, ref != 0)
        assert np.abs(out[b] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("name,precision,rtol", [("c0", "fp64", 1e-11), ("c1", "fp64", 1e-11),
                                                 ("c3", "fp64", 1e-10), ("c1", "mixed", 1e-8),
                                                 ("c3", "mixed", 1e-8)])
def test_newton_step_matches_dense_solve(name, precision, rtol, device):
    from paper_2606_07099_amd.pf import PF_EVAL_STEP
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, precision=precision)
    count = min(sc.batch, 8)
    vm, va, tvm, tva = _states(net, device, count, 13)
    out = tpl.evaluate(PF_EVAL_STEP, d["pd"], d["qd"], d["pg"], d["vset"], tvm, tva,
                       count=count).cpu().numpy()
    for b in range(count):
        J = oracle_j1_paper(net, vm[b], va[b])
        F = oracle_f1(net, sc, b, vm[b], va[b])
        ref = np.linalg.solve(J, -F)
        assert np.linalg.norm(out[b] - ref) <= rtol * np.linalg.norm(ref)


@pytest.mark.parametrize("name,precision,rtol", [("c0", "fp64", 1e-11), ("c1", "fp64", 1e-11),
                                                 ("c3", "fp64", 1e-10), ("c1", "mixed", 1e-8)])
def test_adjoint_solve_matches_dense_transposed_solve(name, precision, rtol, device):
    import torch
    from paper_2606_07099_amd.pf import PF_EVAL_ADJOINT
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, precision=precision)
    count = min(sc.batch, 8)
    vm, va, tvm, tva = _states(net, device, count, 14)
    nj = tpl.n_j
    rhs = np.random.default_rng(15).standard_normal((count, nj))
    out = tpl.evaluate(PF_EVAL_ADJOINT, d["pd"], d["qd"], d["pg"], d["vset"], tvm, tva,
                       rhs=to_dev(rhs, device), count=count).cpu().numpy()
    for b in range(count):
        J = oracle_j1_paper(net, vm[b], va[b])
        ref = np.linalg.solve(J.T, rhs[b])
        assert np.linalg.norm(out[b] - ref) <= rtol * np.linalg.norm(ref)


# ---------------------------------------------------------------- end to end

def _check_solution(net, sc, which, res, oracle, tol, iters_slack=0):
    vm, va, iters, status, fn = (x.cpu().numpy() for x in res)
    for k, b in enumerate(which):
        assert status[b] == oracle.status[k], (b, status[b], oracle.status[k])
        if oracle.status[k] != 0:
            continue
        assert np.abs(vm[b] - oracle.vm[k]).max() <= 1e-8, b
        assert np.abs(va[b] - oracle.va[k]).max() <= 1e-8, b
        assert fn[b] < tol
        d_it = int(iters[b]) - int(oracle.iters[k])
        if iters_slack == 0:
            assert d_it == 0 or tie_band(oracle.histories[k], iters[b], oracle.iters[k], tol), b
        else:
            assert 0 <= d_it <= iters_slack or tie_band(oracle.histories[k], iters[b],
                                                         oracle.iters[k], tol), b


@pytest.mark.parametrize("name,n_check", [("c0", 64), ("c1", 48), ("c3", 12), ("c2", 6)])
def test_newton_fp64_matches_oracle(name, n_check, device):
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device)
    res = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    torch.cuda.synchronize()
    which = np.unique(np.linspace(0, sc.batch - 1, n_check).astype(int))
    oracle = newton_batch(ybus_of(net), net.bus_type, sc, tol=tol, which=which)
    _check_solution(net, sc, which, res, oracle, tol)
    status = res[3].cpu().numpy()
    assert np.all(status == 0)


@pytest.mark.parametrize("name,n_check", [("c1", 48), ("c3", 12), ("c2", 6)])
def test_newton_mixed_precision_matches_oracle(name, n_check, device):
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, precision="mixed")
    res = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    torch.cuda.synchronize()
    which = np.unique(np.linspace(0, sc.batch - 1, n_check).astype(int))
    oracle = newton_batch(ybus_of(net), net.bus_type, sc, tol=tol, which=which)
    _check_solution(net, sc, which, res, oracle, tol, iters_slack=1)
    assert np.all(res[3].cpu().numpy() == 0)
    assert np.all(res[4].cpu().numpy() < tol)


@pytest.mark.parametrize("name,refine,adaptive,n_check", [("c1", 2, True, 48), ("c1", 0, False, 48),
                                                          ("c3", 2, True, 12), ("c2", 2, True, 6),
                                                          ("c2", 0, False, 6)])
def test_mixed_adaptive_and_unrefined_match_oracle(name, refine, adaptive, n_check, device):
    """Adaptive refinement (inexact-Newton forcing term) and no refinement at
    all (FP32 steps corrected only by the FP64 outer Newton loop): the
    convergence test stays on the FP64 mismatch, so the solutions match the
    FP64 oracle to the same bar, at most one extra Newton update."""
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, precision="mixed", refine_steps=refine,
                                               refine_adaptive=adaptive)
    res = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    torch.cuda.synchronize()
    which = np.unique(np.linspace(0, sc.batch - 1, n_check).astype(int))
    oracle = newton_batch(ybus_of(net), net.bus_type, sc, tol=tol, which=which)
    _check_solution(net, sc, which, res, oracle, tol, iters_slack=1)
    assert np.all(res[3].cpu().numpy() == 0)
    assert np.all(res[4].cpu().numpy() < tol)


@pytest.mark.parametrize("name,precision,refine,adaptive,n_check",
                         [("c1", "fp64", 2, False, 48), ("c1", "mixed", 2, False, 48),
                          ("c1", "mixed", 0, False, 48), ("c3", "mixed", 2, True, 12),
                          ("c2", "fp64", 2, False, 4), ("c2", "mixed", 0, False, 4)])
def test_paper_uniform_perturbation_scenarios_match_oracle(name, precision, refine, adaptive, n_check,
                                                            device):
    """The paper's own scenario set: independent uniform +-10% perturbations
    of every PQ load's P and Q (eq. pdqd_perturb).  FP64 to the exact bar,
    the mixed-precision variants with at most one extra update."""
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, precision=precision, refine_steps=refine,
                                               refine_adaptive=adaptive, scenario_mode="uniform10",
                                               batch=256 if name == "c2" else None)
    res = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    torch.cuda.synchronize()
    which = np.unique(np.linspace(0, sc.batch - 1, n_check).astype(int))
    oracle = newton_batch(ybus_of(net), net.bus_type, sc, tol=tol, which=which)
    _check_solution(net, sc, which, res, oracle, tol, iters_slack=0 if precision == "fp64" else 1)
    assert np.all(res[3].cpu().numpy() == 0)


def test_large_grid_solution_satisfies_the_equations(device):
    """9241-bus grid, batch 256: every scenario converges and the oracle's own
    mismatch at the returned voltages is below the tolerance (a property that
    holds at any size; the dense oracle Newton is too slow at this size)."""
    import torch
    from oracle.newton import Index, mismatch, specified
    spec, net, sc, tpl, d, tol = make_gpu_case("c4", device, precision="mixed")
    vm, va, iters, status, fn = (x.cpu().numpy() for x in tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"]))
    assert np.all(status == 0) and np.all(fn < tol)
    Y = ybus_of(net)
    idx = Index.of(net.bus_type)
    for b in (0, 97, 255):
        p, q = specified(sc.pd[b], sc.qd[b], sc.pg[b], net.bus_type)
        F = mismatch(Y, vm[b] * np.exp(1j * va[b]), p, q, idx)
        assert np.abs(F).max() < 1.001 * tol


# ---------------------------------------------------------------- structure / determinism

def test_batch_independence_and_determinism(device):
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case("c1", device, batch=64)
    r1 = [x.clone() for x in tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])]
    r2 = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    for a, b in zip(r1, r2):
        assert torch.equal(a, b)
    # scenario 37 alone (batch of one) equals scenario 37 inside the batch, bitwise
    from paper_2606_07099_amd import PFTemplate
    one = PFTemplate.from_network(net, 1, tol=tol)
    r3 = one.solve(*(d[k][37:38].contiguous() for k in ("pd", "qd", "pg", "vset")))
    assert torch.equal(r3[0][0], r1[0][37]) and torch.equal(r3[1][0], r1[1][37])
    assert int(r3[2][0]) == int(r1[2][37])


def test_max_iter_zero_and_zero_injection(device):
    import torch
    from paper_2606_07099_amd import PFTemplate
    spec, net, sc, tpl, d, tol = make_gpu_case("c0", device, batch=4, max_iter=0)
    vm, va, iters, status, fn = (x.cpu().numpy() for x in tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"]))
    assert np.all(status == 1) and np.all(iters == 0)
    # no load, no charging, unit setpoints: the flat start is the solution
    from paper_2606_07099_amd import ybus_from_branches
    ip, ix, g, b = ybus_from_branches(net.n_bus, net.f, net.t, net.r, net.x, np.zeros_like(net.bc))
    t0 = PFTemplate(net.n_bus, net.bus_type, ip, ix, g, b, 4)
    z = torch.zeros_like(d["pd"][:4].contiguous())
    vm, va, iters, status, fn = (x.cpu().numpy() for x in t0.solve(z, z, z, torch.ones_like(z)))
    assert np.all(status == 0) and np.all(iters == 0)
    assert np.all(vm == 1.0) and np.all(va == 0.0)


def test_adjoint_requires_a_solve(device):
    import torch
    from paper_2606_07099_amd import PFError
    spec, net, sc, tpl, d, tol = make_gpu_case("c0", device, batch=4)
    g = torch.zeros_like(d["pd"])
    with pytest.raises(PFError):
        tpl.adjoint(g, g)
    spec, net, sc, tpl2, d, tol = make_gpu_case("c0", device, batch=4, keep_factors=False)
    tpl2.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    with pytest.raises(PFError):
        tpl2.adjoint(g, g)


@pytest.mark.parametrize("batch", [1, 3, 1023])
def test_ragged_and_single_scenario_batches(batch, device):
    """LDS-resident slices of 4 scenarios with a ragged last slice (and a
    batch of one): every scenario still matches the oracle."""
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case("c1", device, batch=batch, precision="mixed")
    assert tpl.info()["lds_resident"] == 1
    res = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    torch.cuda.synchronize()
    which = np.unique(np.array([0, batch // 2, batch - 1]))
    oracle = newton_batch(ybus_of(net), net.bus_type, sc, tol=tol, which=which)
    _check_solution(net, sc, which, res, oracle, tol, iters_slack=1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_admittance_branch_gives_zero_pivot_status(device, precision):
    """A branch whose admittance entries are present in the pattern but zero
    leaves its far bus with an all-zero Jacobian block: the factorisation
    reports status 3 (zero pivot) for that scenario, and the dense oracle
    Jacobian is exactly singular there.  Two block rows: no dense tail, so
    this covers the pivot test of the level-scheduled factorisation."""
    import torch
    from paper_2606_07099_amd import PFTemplate
    # slack 0 -- PQ 1 -- PQ 2, the 1-2 branch with zero admittance
    y01 = 1.0 / complex(0.01, 0.1)
    Yd = np.zeros((3, 3), complex)
    Yd[0, 0] = Yd[1, 1] = y01
    Yd[0, 1] = Yd[1, 0] = -y01
    indptr = np.array([0, 2, 5, 7], np.int32)
    indices = np.array([0, 1, 0, 1, 2, 1, 2], np.int32)
    g = np.array([Yd[r, c].real for r, c in zip([0, 0, 1, 1, 1, 2, 2], indices)])
    b = np.array([Yd[r, c].imag for r, c in zip([0, 0, 1, 1, 1, 2, 2], indices)])
    bt = np.array([2, 0, 0], np.int32)
    tpl = PFTemplate(3, bt, indptr, indices, g, b, 2, tol=1e-10, precision=precision)
    pd = torch.tensor([[0.0, 0.3, 0.0], [0.0, 0.3, 0.2]], dtype=torch.float64, device=device)
    qd = 0.1 * pd
    vset = torch.ones_like(pd)
    vm, va, iters, status, fn = (x.cpu().numpy() for x in tpl.solve(pd, qd, None, vset))
    assert status[0] == 3 and status[1] == 3
    from oracle.newton import Index, j1
    J = j1(Yd, np.ones(3, complex), Index.of(bt))
    assert np.linalg.matrix_rank(J) < J.shape[0]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_pivot_inside_the_dense_tail(device, precision):
    """A path slack - 1 - 2 - 3 - 4 - 5 whose last branch has zero admittance:
    the five block rows form a chain of single-row levels, all of them in
    the dense tail, and the far bus's block is exactly zero, so the tail's
    pivot test (run once after its elimination) must report status 3 for
    every scenario; the dense oracle Jacobian is singular."""
    import torch
    from paper_2606_07099_amd import PFTemplate
    n = 6
    y = 1.0 / complex(0.01, 0.1)
    Yd = np.zeros((n, n), complex)
    for i in range(n - 2):   # branches (0,1) .. (3,4); (4,5) has zero admittance
        Yd[i, i] += y
        Yd[i + 1, i + 1] += y
        Yd[i, i + 1] -= y
        Yd[i + 1, i] -= y
    rows = [(i, j) for i in range(n) for j in range(n) if abs(i - j) <= 1]
    indptr = np.zeros(n + 1, np.int32)
    for i, _ in rows:
        indptr[i + 1] += 1
    indptr = np.cumsum(indptr).astype(np.int32)
    indices = np.array([j for _, j in rows], np.int32)
    g = np.array([Yd[i, j].real for i, j in rows])
    b = np.array([Yd[i, j].imag for i, j in rows])
    bt = np.array([2, 0, 0, 0, 0, 0], np.int32)
    tpl = PFTemplate(n, bt, indptr, indices, g, b, 3, tol=1e-10, precision=precision)
    pd = torch.tensor([[0.0, 0.1, 0.1, 0.1, 0.1, 0.0],
                       [0.0, 0.2, 0.1, 0.0, 0.1, 0.0],
                       [0.0, 0.0, 0.0, 0.0, 0.0, 0.0]], dtype=torch.float64, device=device)
    qd = 0.1 * pd
    vset = torch.ones_like(pd)
    vm, va, iters, status, fn = (x.cpu().numpy() for x in tpl.solve(pd, qd, None, vset))
    # the zero-load scenario converges at the flat start, before any factorisation
    assert status.tolist() == [3, 3, 0]
    from oracle.newton import Index, j1
    J = j1(Yd, np.ones(n, complex), Index.of(bt))
    assert np.linalg.matrix_rank(J) < J.shape[0]


# ---------------------------------------------------------------- properties at full size

@pytest.mark.parametrize("name,precision", [("c2", "fp64"), ("c2", "mixed"), ("c4", "fp64"), ("c4", "mixed")])
def test_adjoint_dot_product_identity_at_full_size(name, precision, device):
    """<lambda, J1 dz> = <J1^T lambda, dz> for the library's own Newton step
    (J1 dz = -F1) and adjoint solve (J1^T lambda = rhs) at the same states, on
    every scenario of the full batch: <lambda, F1> = -<rhs, dz> (a property
    that holds at any size, where the dense oracle cannot follow)."""
    import torch
    from paper_2606_07099_amd.pf import PF_EVAL_ADJOINT, PF_EVAL_MISMATCH, PF_EVAL_STEP
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, precision=precision)
    count = sc.batch
    rng = np.random.default_rng(31)
    vm = rng.uniform(0.97, 1.03, (count, net.n_bus))
    va = rng.uniform(-0.05, 0.05, (count, net.n_bus))
    va[:, net.bus_type == 2] = 0.0
    tvm, tva = to_dev(vm, device), to_dev(va, device)
    args = (d["pd"], d["qd"], d["pg"], d["vset"], tvm, tva)
    F = tpl.evaluate(PF_EVAL_MISMATCH, *args, count=count).cpu().numpy()
    dz = tpl.evaluate(PF_EVAL_STEP, *args, count=count).cpu().numpy()
    rhs = rng.standard_normal((count, tpl.n_j))
    lam = tpl.evaluate(PF_EVAL_ADJOINT, *args, rhs=to_dev(rhs, device), count=count).cpu().numpy()
    torch.cuda.synchronize()
    lhs = np.einsum("bi,bi->b", lam, F)
    rhv = -np.einsum("bi,bi->b", rhs, dz)
    scale = np.linalg.norm(lam, axis=1) * np.linalg.norm(F, axis=1)
    assert np.all(np.abs(lhs - rhv) <= 1e-9 * scale), np.max(np.abs(lhs - rhv) / scale)


def test_gradient_matches_directional_differences_on_every_scenario(device):
    """The 300-bus batch of 2048, FP64: for a random load direction per
    scenario, central differences of the library's own forward solves
    (Richardson-extrapolated over h and h/2, error O(h^4)) agree with the
    library's adjoint gradient on every scenario, relative to the natural
    scale |grad| |direction|."""
    import torch
    spec, net, sc, tpl, d, tol = make_gpu_case("c3", device, precision="fp64", tol=1e-12, max_iter=30)
    B, n = sc.batch, net.n_bus
    rng = np.random.default_rng(17)
    dirn = np.zeros((B, n))
    pq = net.bus_type == 0
    dirn[:, pq] = rng.standard_normal((B, int(pq.sum())))
    ddir = to_dev(dirn, device)

    def loss_at(step):
        vm, va, _, st, _ = tpl.solve(d["pd"] + step * ddir, d["qd"], d["pg"], d["vset"])
        assert int((st != 0).sum()) == 0
        return ((vm - 1.0) ** 2).sum(dim=1) + 0.1 * (va ** 2).sum(dim=1)

    h = 2e-4
    fd_h = (loss_at(h) - loss_at(-h)) / (2 * h)
    fd_h2 = (loss_at(h / 2) - loss_at(-h / 2)) / h
    fd = ((4.0 * fd_h2 - fd_h) / 3.0).cpu().numpy()
    vm, va, _, s0, _ = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    g_pd, g_qd, g_pg, g_vs = tpl.adjoint((2.0 * (vm - 1.0)).contiguous(), (0.2 * va).contiguous())
    torch.cuda.synchronize()
    assert int((s0 != 0).sum()) == 0
    ad = (g_pd * ddir).sum(dim=1).cpu().numpy()
    scale = np.linalg.norm(g_pd.cpu().numpy(), axis=1) * np.linalg.norm(dirn, axis=1)
    err = np.abs(fd - ad) / scale
    assert np.all(err <= 1e-6), (err.max(), int(err.argmax()))
