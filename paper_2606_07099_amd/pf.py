"""Python handle on a power-flow template (ctypes marshalling only).

Torch is used for device memory and streams: batch arrays are contiguous
float64 CUDA tensors of shape [batch, n_bus]; calls are enqueued on the
current torch stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (PFError, PFOptions, PFStats, check, lib, PF_FP64, PF_MIXED, PF_EVAL_ADJOINT,
                   PF_EVAL_FILL, PF_EVAL_JACOBIAN, PF_EVAL_MISMATCH, PF_EVAL_STEP, PF_OP_BASE, PF_OP_J1,
                   PF_OP_J1T, PF_OP_J2T, PF_OP_J3T)

_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32P)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_F64P)


def ybus_from_branches(n_bus, f, t, r, x, bc):
    """Y_bus CSR (indptr, indices, g, b) of a pi-model branch list, by the library."""
    L = lib()
    f_, fp = _i32(f)
    t_, tp = _i32(t)
    r_, rp = _f64(r)
    x_, xp = _f64(x)
    b_, bp = _f64(bc)
    m = int(f_.shape[0])
    cap = 4 * m + n_bus
    indptr = np.zeros(n_bus + 1, np.int32)
    ind = np.zeros(cap, np.int32)
    g = np.zeros(cap)
    b = np.zeros(cap)
    nnz = ctypes.c_int32(0)
    check(L.pf_ybus_from_branches(n_bus, m, fp, tp, rp, xp, bp, indptr.ctypes.data_as(_I32P),
                                  ind.ctypes.data_as(_I32P), g.ctypes.data_as(_F64P),
                                  b.ctypes.data_as(_F64P), cap, ctypes.byref(nnz)))
    k = nnz.value
    return indptr, ind[:k].copy(), g[:k].copy(), b[:k].copy()


def symbolic_analyze(n_bus, bus_type, indptr, indices):
    """Host-only symbolic statistics and bus elimination order (no GPU needed)."""
    L = lib()
    st = PFStats()
    bt, btp = _i32(bus_type)
    ip, ipp = _i32(indptr)
    ix, ixp = _i32(indices)
    order = np.zeros(n_bus - 1, np.int32)
    check(L.pf_symbolic_analyze(n_bus, btp, ipp, ixp, ctypes.byref(st), order.ctypes.data_as(_I32P)))
    return st.as_dict(), order


def operator_pattern(n_bus, bus_type, indptr, indices, which):
    """One scenario's CSR pattern of operator ``which`` (PF_OP_*), host only:
    dict with n_rows, n_cols, indptr, indices and pos (the base-to-operator
    position map, -1 where unused)."""
    L = lib()
    bt, btp = _i32(bus_type)
    ip, ipp = _i32(indptr)
    ix, ixp = _i32(indices)
    nr, nc, nz, nzb = (ctypes.c_int32(0) for _ in range(4))
    null = ctypes.cast(None, _I32P)
    check(L.pf_operator_pattern(int(n_bus), btp, ipp, ixp, int(which), ctypes.byref(nr), ctypes.byref(nc),
                                ctypes.byref(nz), ctypes.byref(nzb), null, null, null))
    out_ptr = np.zeros(nr.value + 1, np.int32)
    out_ix = np.zeros(nz.value, np.int32)
    out_pos = np.zeros(nzb.value, np.int32)
    check(L.pf_operator_pattern(int(n_bus), btp, ipp, ixp, int(which), ctypes.byref(nr), ctypes.byref(nc),
                                ctypes.byref(nz), ctypes.byref(nzb), out_ptr.ctypes.data_as(_I32P),
                                out_ix.ctypes.data_as(_I32P), out_pos.ctypes.data_as(_I32P)))
    return {"n_rows": nr.value, "n_cols": nc.value, "indptr": out_ptr, "indices": out_ix, "pos": out_pos}


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class PFTemplate:
    """A network + batch size: the one-time symbolic analysis and the device
    workspace of ``pf_template_build``."""

    def __init__(self, n_bus, bus_type, indptr, indices, g, b, batch, *, tol=1e-8, max_iter=20,
                 precision="fp64", refine_steps=2, keep_factors=True, block_threads=0,
                 refine_adaptive=False):
        L = lib()
        opt = PFOptions()
        L.pf_default_options(ctypes.byref(opt))
        opt.tol = float(tol)
        opt.max_iter = int(max_iter)
        opt.precision = {"fp64": PF_FP64, "mixed": PF_MIXED}[precision]
        opt.refine_steps = int(refine_steps)
        opt.keep_factors = 1 if keep_factors else 0
        opt.block_threads = int(block_threads)
        opt.refine_adaptive = 1 if refine_adaptive else 0
        self.n_bus = int(n_bus)
        self.batch = int(batch)
        self.precision = precision
        self._bt, btp = _i32(bus_type)
        self._ip, ipp = _i32(indptr)
        self._ix, ixp = _i32(indices)
        self._g, gp = _f64(g)
        self._b, bp = _f64(b)
        import torch
        self.device = torch.cuda.current_device() if torch.cuda.is_available() else 0
        h = ctypes.c_void_p()
        check(L.pf_template_build(self.n_bus, btp, ipp, ixp, gp, bp, self.batch, ctypes.byref(opt),
                                  ctypes.byref(h)))
        self._h = h
        self._solve_id = 0

    @classmethod
    def from_network(cls, net, batch, **kw):
        indptr, ind, g, b = ybus_from_branches(net.n_bus, net.f, net.t, net.r, net.x, net.bc)
        return cls(net.n_bus, net.bus_type, indptr, ind, g, b, batch, **kw)

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pf_template_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        st = PFStats()
        check(lib().pf_template_info(self._h, ctypes.byref(st)))
        return st.as_dict()

    @property
    def n_j(self) -> int:
        return self.info()["n_j"]

    # ------------------------------------------------------------------
    def _check(self, name, x, rows=None, cols=None):
        """A float64 contiguous CUDA tensor on the template's device with at
        least ``rows`` rows of ``cols`` columns (default: batch x n_bus)."""
        import torch
        rows = self.batch if rows is None else rows
        cols = self.n_bus if cols is None else cols
        if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if x.device.index != self.device:
            raise ValueError(f"{name} is on {x.device}, the template on cuda:{self.device}")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if x.dim() != 2 or x.shape[0] < rows or x.shape[1] != cols:
            raise ValueError(f"{name} must have shape [{rows}, {cols}], got {tuple(x.shape)}")
        return ctypes.c_void_p(x.data_ptr())

    def solve(self, pd, qd, pg, vset, *, out=None, stream=None):
        """Newton solve of the whole batch from the flat start.  Returns
        (vm, va, iters, status, final_mismatch) as device tensors."""
        import torch
        dev = pd.device
        if out is None:
            vm = torch.empty((self.batch, self.n_bus), dtype=torch.float64, device=dev)
            va = torch.empty_like(vm)
            iters = torch.empty(self.batch, dtype=torch.int32, device=dev)
            status = torch.empty_like(iters)
            fn = torch.empty(self.batch, dtype=torch.float64, device=dev)
        else:
            vm, va, iters, status, fn = out
        for nm, x, dt in (("iters", iters, torch.int32), ("status", status, torch.int32),
                          ("final_mismatch", fn, torch.float64)):
            if (not isinstance(x, torch.Tensor) or x.dtype != dt or not x.is_cuda or not x.is_contiguous()
                    or x.device.index != self.device or x.numel() < self.batch):
                raise ValueError(f"{nm} must be a contiguous {dt} CUDA tensor of {self.batch} elements "
                                 f"on cuda:{self.device}")
        args = [self._check("pd", pd), self._check("qd", qd),
                self._check("pg", pg) if pg is not None else ctypes.c_void_p(0),
                self._check("vset", vset), self._check("vm", vm), self._check("va", va)]
        check(lib().pf_solve_batch(self._h, *args, ctypes.c_void_p(iters.data_ptr()),
                                   ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(fn.data_ptr()),
                                   _stream_ptr(stream)))
        self._solve_id += 1
        return vm, va, iters, status, fn

    def adjoint(self, g_vm, g_va, *, stream=None):
        """Gradients (g_pd, g_qd, g_pg, g_vset) of the most recent solve."""
        import torch
        outs = [torch.empty_like(g_vm) for _ in range(4)]
        check(lib().pf_adjoint_batch(self._h, self._check("g_vm", g_vm), self._check("g_va", g_va),
                                     *[ctypes.c_void_p(o.data_ptr()) for o in outs],
                                     _stream_ptr(stream)))
        return tuple(outs)

    def recover(self, pd, qd, pg, vm, va, *, stream=None):
        """Step-2 generation block (pg_out, qg_out) at the solution (vm, va)."""
        import torch
        pg_out = torch.empty_like(vm)
        qg_out = torch.empty_like(vm)
        check(lib().pf_recover_batch(self._h, self._check("pd", pd), self._check("qd", qd),
                                     self._check("pg", pg) if pg is not None else ctypes.c_void_p(0),
                                     self._check("vm", vm), self._check("va", va),
                                     ctypes.c_void_p(pg_out.data_ptr()),
                                     ctypes.c_void_p(qg_out.data_ptr()), _stream_ptr(stream)))
        return pg_out, qg_out

    def adjoint_completed(self, g_vm, g_va, g_pg_out=None, g_qg_out=None, *, stream=None):
        """Gradients (g_pd, g_qd, g_pg, g_vset) of the most recent solve for a
        loss on (vm, va) and on the recovered generation (pg_out, qg_out)."""
        import torch
        outs = [torch.empty_like(g_vm) for _ in range(4)]
        opt = [self._check(k, v) if v is not None else ctypes.c_void_p(0)
               for k, v in (("g_pg_out", g_pg_out), ("g_qg_out", g_qg_out))]
        check(lib().pf_adjoint_completed_batch(self._h, self._check("g_vm", g_vm),
                                               self._check("g_va", g_va), *opt,
                                               *[ctypes.c_void_p(o.data_ptr()) for o in outs],
                                               _stream_ptr(stream)))
        return tuple(outs)

    def block_pattern(self):
        """(row_bus, col_bus) of every 2x2 block of L+U in the library's order."""
        nnzb = self.info()["nnzb_lu"]
        rb = np.zeros(nnzb, np.int32)
        cb = np.zeros(nnzb, np.int32)
        check(lib().pf_template_block_pattern(self._h, rb.ctypes.data_as(_I32P), cb.ctypes.data_as(_I32P)))
        return rb, cb

    def operator_pattern(self, which):
        """One scenario's CSR pattern of operator ``which`` (see :func:`operator_pattern`)."""
        return operator_pattern(self.n_bus, self._bt, self._ip, self._ix, which)

    def operator(self, which, vm, va, *, out=None, stream=None):
        """Batch-global operator ``which`` at the states (vm, va) [count, n_bus]:
        a torch sparse CSR tensor that embeds each scenario's block on the
        diagonal (eq. BDE_global).  Its pattern is built once per (operator,
        count) and cached; pass a previous result as ``out`` to refresh its
        value array in place instead of allocating a new one."""
        import torch
        count = int(vm.shape[0])
        self._check("vm", vm, count)
        self._check("va", va, count)
        if tuple(va.shape) != tuple(vm.shape):
            raise ValueError("vm and va must have the same shape [count, n_bus]")
        cache = self.__dict__.setdefault("_op_cache", {})
        key = (int(which), count, vm.device)
        if key not in cache:   # the batch-global pattern, expanded by the library
            pat = self.operator_pattern(which)
            nr, nc, nnz = pat["n_rows"], pat["n_cols"], int(pat["indices"].size)
            crow = torch.empty(count * nr + 1, dtype=torch.int64, device=vm.device)
            col = torch.empty(max(count * nnz, 1), dtype=torch.int64, device=vm.device)
            check(lib().pf_operator_bde_csr(self._h, int(which), count, ctypes.c_void_p(crow.data_ptr()),
                                            ctypes.c_void_p(col.data_ptr()), _stream_ptr(stream)))
            cache[key] = (crow, col[:count * nnz], nnz, (count * nr, count * nc))
        crow, col, nnz, shape = cache[key]
        if out is not None:
            values = out.values()
            if values.numel() != count * nnz or not values.is_contiguous():
                raise ValueError("out does not match this operator and batch")
        else:
            values = torch.empty(count * nnz, dtype=torch.float64, device=vm.device)
        check(lib().pf_operator_values(self._h, int(which), count, ctypes.c_void_p(vm.data_ptr()),
                                       ctypes.c_void_p(va.data_ptr()), ctypes.c_void_p(values.data_ptr()),
                                       _stream_ptr(stream)))
        if out is not None:
            return out
        return torch.sparse_csr_tensor(crow, col, values, size=shape)

    def evaluate(self, mode, pd, qd, pg, vset, vm, va, rhs=None, count=None, *, stream=None):
        """Kernel-level evaluation at a given state (see ``pf_eval_batch``)."""
        import torch
        count = self.batch if count is None else int(count)
        nj = self.n_j
        shape = {PF_EVAL_JACOBIAN: (count, nj, nj),
                 PF_EVAL_FILL: (count, 4 * self.info()["nnzb_lu"])}.get(mode, (count, nj))
        out = torch.empty(shape, dtype=torch.float64, device=vm.device)
        r = ctypes.c_void_p(0)
        if rhs is not None:
            r = self._check("rhs", rhs, count, nj)
        elif mode == PF_EVAL_ADJOINT:
            raise ValueError("PF_EVAL_ADJOINT needs rhs [count, n_j]")
        check(lib().pf_eval_batch(self._h, int(mode), count,
                                  self._check("pd", pd, count), self._check("qd", qd, count),
                                  self._check("pg", pg, count) if pg is not None else ctypes.c_void_p(0),
                                  self._check("vset", vset, count), self._check("vm", vm, count),
                                  self._check("va", va, count), r, ctypes.c_void_p(out.data_ptr()),
                                  _stream_ptr(stream)))
        return out


__all__ = ["PFTemplate", "ybus_from_branches", "symbolic_analyze", "operator_pattern", "PFError",
           "PF_EVAL_MISMATCH", "PF_EVAL_JACOBIAN", "PF_EVAL_STEP", "PF_EVAL_ADJOINT", "PF_EVAL_FILL", "PF_OP_BASE",
           "PF_OP_J1", "PF_OP_J1T", "PF_OP_J2T", "PF_OP_J3T"]
