"""Host-side checks of the C-ABI library (no GPU): exports, Y_bus assembly,
symbolic analysis, input validation."""
import ctypes
import os
import re

import numpy as np
import pytest

from gen.grids import SPECS, make_network, PQ, PV, SLACK
from oracle.ybus import ybus_of

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sable_pf.h")


@pytest.fixture(scope="module")
def L():
    from paper_2606_07099_amd import _lib
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_exported_api():
    from paper_2606_07099_amd._lib import EXPORTED
    assert sorted(EXPORTED) == declared_functions()


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_default_options(L):
    from paper_2606_07099_amd._lib import PFOptions
    o = PFOptions()
    L.pf_default_options(ctypes.byref(o))
    assert (o.tol, o.max_iter, o.precision, o.refine_steps, o.keep_factors, o.block_threads,
            o.refine_adaptive) == (1e-8, 20, 0, 2, 1, 0, 0)


@pytest.mark.parametrize("name", ["c0", "c1", "c3"])
def test_ybus_from_branches_matches_oracle(name):
    from paper_2606_07099_amd import ybus_from_branches
    net = make_network(SPECS[name])
    ip, ix, g, b = ybus_from_branches(net.n_bus, net.f, net.t, net.r, net.x, net.bc)
    Yd = np.zeros((net.n_bus, net.n_bus), complex)
    for i in range(net.n_bus):
        assert np.all(np.diff(ix[ip[i]:ip[i + 1]]) > 0)
        Yd[i, ix[ip[i]:ip[i + 1]]] = g[ip[i]:ip[i + 1]] + 1j * b[ip[i]:ip[i + 1]]
    Y = ybus_of(net)
    assert np.abs(Yd - Y).max() <= 1e-12 * np.abs(Y).max()
    assert set(zip(*np.nonzero(Y))) <= set(zip(*np.nonzero(Yd)))


def _bus_graph(net):
    n = net.n_bus
    adj = [set() for _ in range(n)]
    for a, c in zip(net.f, net.t):
        adj[a].add(c)
        adj[c].add(a)
    return adj


def _reference_fill(net, order):
    """Symbolic elimination written directly: eliminate the buses in `order`
    on a dense boolean matrix and count the block pattern of L+U."""
    slack = int(np.flatnonzero(net.bus_type == SLACK)[0])
    nb = net.n_bus - 1
    pos = {bus: r for r, bus in enumerate(order)}
    A = np.zeros((nb, nb), bool)
    for bus, nbrs in enumerate(_bus_graph(net)):
        if bus == slack:
            continue
        A[pos[bus], pos[bus]] = True
        for m in nbrs:
            if m != slack:
                A[pos[bus], pos[m]] = True
    for k in range(nb):
        rows = np.flatnonzero(A[k + 1:, k]) + k + 1
        cols = np.flatnonzero(A[k, k + 1:]) + k + 1
        A[np.ix_(rows, cols)] = True
    return A


@pytest.mark.parametrize("name", ["c0", "c1", "c3", "c2"])
def test_symbolic_pattern_matches_dense_elimination(name):
    from paper_2606_07099_amd import symbolic_analyze, ybus_from_branches
    net = make_network(SPECS[name])
    ip, ix, g, b = ybus_from_branches(net.n_bus, net.f, net.t, net.r, net.x, net.bc)
    st, order = symbolic_analyze(net.n_bus, net.bus_type, ip, ix)
    slack = int(np.flatnonzero(net.bus_type == SLACK)[0])
    assert sorted(order.tolist()) == [i for i in range(net.n_bus) if i != slack]
    A = _reference_fill(net, order)
    assert st["nnzb_lu"] == int(A.sum())
    nu = np.where(net.bus_type[order] == PQ, 2, 1)
    assert st["nnz_lu"] == int((A * nu[:, None] * nu[None, :]).sum())
    # J1's own pattern (no fill) counted from the network
    nnz_j1 = 0
    for bus, nbrs in enumerate(_bus_graph(net)):
        if bus == slack:
            continue
        nb_u = 2 if net.bus_type[bus] == PQ else 1
        for m in list(nbrs) + [bus]:
            if m != slack:
                nnz_j1 += nb_u * (2 if net.bus_type[m] == PQ else 1)
    assert st["nnz_j1"] == nnz_j1
    assert st["n_j"] == (net.n_bus - 1) + int((net.bus_type == PQ).sum())
    assert 1.0 <= st["fill_ratio"] < 3.0


def test_minimum_degree_beats_natural_order_on_fill():
    from paper_2606_07099_amd import symbolic_analyze, ybus_from_branches
    net = make_network(SPECS["c3"])
    ip, ix, g, b = ybus_from_branches(net.n_bus, net.f, net.t, net.r, net.x, net.bc)
    st, order = symbolic_analyze(net.n_bus, net.bus_type, ip, ix)
    natural = [i for i in range(net.n_bus) if net.bus_type[i] != SLACK]
    assert st["nnzb_lu"] < _reference_fill(net, natural).sum()


def _analyze(bt, f, t, n):
    from paper_2606_07099_amd import symbolic_analyze, ybus_from_branches
    m = len(f)
    ip, ix, g, b = ybus_from_branches(n, f, t, np.full(m, 0.01), np.full(m, 0.1), np.zeros(m))
    return symbolic_analyze(n, np.array(bt, np.int32), ip, ix)


def test_rejects_bad_topologies():
    from paper_2606_07099_amd._lib import PFError, PF_ETOPOLOGY, PF_EINVAL
    with pytest.raises(PFError) as e:       # two slack buses
        _analyze([SLACK, SLACK, PQ], [0, 1], [1, 2], 3)
    assert e.value.code == PF_ETOPOLOGY
    with pytest.raises(PFError) as e:       # no slack
        _analyze([PQ, PV, PQ], [0, 1], [1, 2], 3)
    assert e.value.code == PF_ETOPOLOGY
    with pytest.raises(PFError) as e:       # isolated bus 3
        _analyze([SLACK, PQ, PQ, PQ], [0, 1], [1, 2], 4)
    assert e.value.code == PF_ETOPOLOGY
    with pytest.raises(PFError) as e:       # bad bus type
        _analyze([SLACK, 7, PQ], [0, 1], [1, 2], 3)
    assert e.value.code == PF_EINVAL


def test_ybus_rejects_self_loops_and_small_capacity(L):
    from paper_2606_07099_amd import ybus_from_branches
    from paper_2606_07099_amd._lib import PFError
    with pytest.raises(PFError):
        ybus_from_branches(3, np.array([0, 1]), np.array([1, 1]), np.ones(2) * 0.01, np.ones(2) * 0.1,
                           np.zeros(2))
    I32 = ctypes.POINTER(ctypes.c_int32)
    F64 = ctypes.POINTER(ctypes.c_double)
    f = np.array([0, 1], np.int32)
    t = np.array([1, 2], np.int32)
    r = np.full(2, 0.01)
    ip = np.zeros(4, np.int32)
    ix = np.zeros(2, np.int32)
    gg = np.zeros(2)
    nnz = ctypes.c_int32(0)
    rc = L.pf_ybus_from_branches(3, 2, f.ctypes.data_as(I32), t.ctypes.data_as(I32), r.ctypes.data_as(F64),
                                 r.ctypes.data_as(F64), r.ctypes.data_as(F64), ip.ctypes.data_as(I32),
                                 ix.ctypes.data_as(I32), gg.ctypes.data_as(F64), gg.ctypes.data_as(F64),
                                 2, ctypes.byref(nnz))
    assert rc != 0 and nnz.value == 7


def test_template_build_rejects_empty_batches_and_bad_options(L):
    """Argument checks that run before any device call: an empty batch, a
    bad precision, too many refinement steps and a block size that is not a
    multiple of the wavefront all fail with PF_EINVAL and a message."""
    from paper_2606_07099_amd import PFTemplate
    from paper_2606_07099_amd._lib import PFError, PF_EINVAL
    from paper_2606_07099_amd.pf import ybus_from_branches
    n, f, t = 3, np.array([0, 1]), np.array([1, 2])
    ip, ix, g, b = ybus_from_branches(n, f, t, np.full(2, 0.01), np.full(2, 0.1), np.zeros(2))
    bt = np.array([SLACK, PQ, PQ], np.int32)
    for kw in ({"batch": 0}, {"batch": -3}, {"batch": 4, "refine_steps": 17},
               {"batch": 4, "block_threads": 100}, {"batch": 4, "max_iter": -1}, {"batch": 4, "tol": 0.0}):
        batch = kw.pop("batch")
        with pytest.raises(PFError) as e:
            PFTemplate(n, bt, ip, ix, g, b, batch, **kw)
        assert e.value.code == PF_EINVAL
        assert L.pf_last_error().decode()
