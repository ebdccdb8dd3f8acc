"""pf_operator_values_static: the operator value refresh whose per-bus state
lives in the library's fixed device array instead of an allocated buffer.
Checked against pf_operator_values (the same kernels, so the values must be
identical) on two calls in a row, the second with a smaller batch, on a grid
whose batch fits the fixed array in one piece and on one that needs several
pieces."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import make_gpu_case, random_states, to_dev

pytestmark = pytest.mark.gpu


def _values(tpl, fn, which, vm, va):
    import torch
    from paper_2606_07099_amd._lib import check, lib
    count = int(vm.shape[0])
    nnz = int(tpl.operator_pattern(which)["indices"].size)
    out = torch.full((count * nnz,), float("nan"), dtype=torch.float64, device=vm.device)
    check(getattr(lib(), fn)(tpl._h, int(which), count, ctypes.c_void_p(vm.data_ptr()),
                             ctypes.c_void_p(va.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


@pytest.mark.parametrize("name,counts", [("c1", (64, 16)), ("c2", (1000, 300))])
def test_static_operator_values_match_the_allocating_entry_point(name, counts, device):
    import torch
    from paper_2606_07099_amd.pf import PF_OP_BASE, PF_OP_J1, PF_OP_J1T, PF_OP_J2T, PF_OP_J3T
    spec, net, sc, tpl, d, tol = make_gpu_case(name, device, batch=64 if name == "c1" else 256)
    for call, count in enumerate(counts):
        vm, va = random_states(net, count, 50 + call)
        tvm, tva = to_dev(vm, device), to_dev(va, device)
        for which in (PF_OP_BASE, PF_OP_J1, PF_OP_J1T, PF_OP_J2T, PF_OP_J3T):
            ref = _values(tpl, "pf_operator_values", which, tvm, tva)
            got = _values(tpl, "pf_operator_values_static", which, tvm, tva)
            torch.cuda.synchronize()
            assert not torch.isnan(got).any(), (name, call, which)
            assert torch.equal(got, ref), (name, call, which, (got - ref).abs().max().item())


def test_static_operator_values_reject_bad_arguments(device):
    import torch
    from paper_2606_07099_amd._lib import PF_EINVAL, lib
    spec, net, sc, tpl, d, tol = make_gpu_case("c0", device, batch=4)
    L = lib()
    rc = L.pf_operator_values_static(tpl._h, 1, 4, None, None, None, None)
    assert rc == PF_EINVAL and b"NULL" in L.pf_last_error()
    rc = L.pf_operator_values_static(tpl._h, 9, 0, None, None, None, None)
    assert rc == PF_EINVAL and b"unknown operator" in L.pf_last_error()
