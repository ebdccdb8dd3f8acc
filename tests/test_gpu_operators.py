"""GPU value refresh of the base Jacobian template and of J1, J1^T, J2^T,
J3^T (eq. J_base_block, step1_jacobian, Jstep2_impl, Jstep3_impl; Algorithms
1 and 2) against the oracle's dense operators at random states, and the
batch-global block-diagonal CSR (eq. BDE_global) as a torch sparse tensor."""
import numpy as np
import pytest

from gpu_helpers import random_states, to_dev
from gen.grids import make_case
from oracle.operators import operators
from oracle.ybus import ybus_of

pytestmark = pytest.mark.gpu

OPS = {0: "J", 1: "J1", 2: "J1T", 3: "J2T", 4: "J3T"}


def _dense(pat, values):
    d = np.zeros((pat["n_rows"], pat["n_cols"]))
    rows = np.repeat(np.arange(pat["n_rows"]), np.diff(pat["indptr"]))
    d[rows, pat["indices"]] = values
    return d


@pytest.mark.parametrize("name,count,n_check", [("c0", 40, 40), ("c1", 64, 6), ("c3", 16, 3), ("c2", 8, 2)])
def test_operator_values_match_oracle(name, count, n_check, device):
    import torch
    from paper_2606_07099_amd import PFTemplate
    spec, net, sc = make_case(name, batch=4)
    tpl = PFTemplate.from_network(net, 4)          # count may exceed the template's batch
    vm, va = random_states(net, count, seed=21)
    vm_d, va_d = to_dev(vm, device), to_dev(va, device)
    Y = ybus_of(net)
    for which, key in OPS.items():
        pat = tpl.operator_pattern(which)
        nnz = pat["indices"].size
        A = tpl.operator(which, vm_d, va_d)
        torch.cuda.synchronize()
        vals = A.values().cpu().numpy().reshape(count, nnz)
        for b in np.unique(np.linspace(0, count - 1, n_check).astype(int)):
            ref = operators(Y, net.bus_type, vm[b], va[b])[key]
            ours = _dense(pat, vals[b])
            scale = np.abs(ref).max()
            assert np.abs(ours - ref).max() <= 1e-12 * scale, (key, b)


def test_block_diagonal_embedding_and_in_place_refresh(device):
    import torch
    from paper_2606_07099_amd import PFTemplate
    from paper_2606_07099_amd.pf import PF_OP_J1, PF_OP_J2T
    spec, net, sc = make_case("c0", batch=3)
    tpl = PFTemplate.from_network(net, 3)
    vm, va = random_states(net, 3, seed=4)
    vm_d, va_d = to_dev(vm, device), to_dev(va, device)
    A = tpl.operator(PF_OP_J1, vm_d, va_d)
    Y = ybus_of(net)
    blocks = [operators(Y, net.bus_type, vm[b], va[b])["J1"] for b in range(3)]
    n1 = blocks[0].shape[0]
    D = A.to_dense().cpu().numpy()
    assert D.shape == (3 * n1, 3 * n1)
    for b in range(3):
        for c in range(3):
            blk = D[b * n1:(b + 1) * n1, c * n1:(c + 1) * n1]
            if b == c:
                assert np.abs(blk - blocks[b]).max() <= 1e-12 * np.abs(blocks[b]).max()
            else:
                assert not blk.any()
    # a sparse product with the global operator is the per-scenario product
    x = torch.randn(3 * n1, 1, dtype=torch.float64, device=device)
    yv = (A @ x).cpu().numpy().ravel()
    xs = x.cpu().numpy().ravel()
    for b in range(3):
        assert np.allclose(yv[b * n1:(b + 1) * n1], blocks[b] @ xs[b * n1:(b + 1) * n1], rtol=1e-12, atol=1e-12)
    # refresh at new states into the same value buffer
    vm2, va2 = random_states(net, 3, seed=5)
    ptr = A.values().data_ptr()
    A2 = tpl.operator(PF_OP_J1, to_dev(vm2, device), to_dev(va2, device), out=A)
    torch.cuda.synchronize()
    assert A2 is A and A.values().data_ptr() == ptr
    ref2 = operators(Y, net.bus_type, vm2[1], va2[1])["J1"]
    assert np.abs(A.to_dense().cpu().numpy()[n1:2 * n1, n1:2 * n1] - ref2).max() <= 1e-12 * np.abs(ref2).max()
    # J2^T of the batch: shape (3 * 2 n_bus, 3 * (1 + n_gen))
    B = tpl.operator(PF_OP_J2T, vm_d, va_d)
    ng = int((net.bus_type != 0).sum())
    assert tuple(B.shape) == (3 * 2 * net.n_bus, 3 * (1 + ng))
