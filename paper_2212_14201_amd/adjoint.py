"""Batched adjoint gradients of Pauli-sum expectations (binding of
``qvm_adjoint_expect_grad``) and a ``torch.autograd.Function`` over them."""
from __future__ import annotations

import ctypes

import numpy as np

from .qvm import GateArray, _dt, _gp, _i32p, _u64p, _dp, _vp, check, lib


def _declare():
    L = lib()
    L.qvm_adjoint_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t]
    L.qvm_adjoint_workspace_bytes.restype = ctypes.c_size_t
    L.qvm_adjoint_expect_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _gp,
                                          ctypes.c_size_t, _i32p, ctypes.c_int, _dp,
                                          ctypes.c_size_t, _u64p, _u64p, _dp, _vp, _vp, _vp,
                                          ctypes.c_size_t, _vp, _dp, _dp]
    L.qvm_adjoint_expect_grad.restype = ctypes.c_int
    L.qvm_adjoint_expect_grad_static.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _gp,
                                                 ctypes.c_size_t, _i32p, ctypes.c_int, _dp,
                                                 ctypes.c_size_t, _u64p, _u64p, _dp, _vp, _vp, _vp,
                                                 _dp, _dp]
    L.qvm_adjoint_expect_grad_static.restype = ctypes.c_int
    L.qvm_adjoint_group_count.argtypes = [ctypes.c_int, ctypes.c_int, _gp, ctypes.c_size_t, _i32p,
                                          ctypes.c_int, _i32p]
    L.qvm_adjoint_group_count.restype = ctypes.c_int
    return L


class AdjointProblem:
    """A parameterised circuit and a Pauli-sum observable, with device
    buffers for a batch of states (psi, lambda) allocated once.

    static_workspace: run through ``qvm_adjoint_expect_grad_static``, whose
    workspace is the library's static per-device array (no workspace
    tensor is allocated here)."""

    def __init__(self, n, gates, n_params, xs, zs, cs, batch, dtype="c64", device="cuda",
                 static_workspace=False):
        import torch
        self.n, self.batch, self.n_params = int(n), int(batch), int(n_params)
        self.dtype = dtype
        self.gates = GateArray(gates)
        self.pidx = np.ascontiguousarray([getattr(g, "pidx", -1) for g in gates], dtype=np.int32)
        self.xs = np.ascontiguousarray(xs, dtype=np.uint64)
        self.zs = np.ascontiguousarray(zs, dtype=np.uint64)
        self.cs = np.ascontiguousarray(cs, dtype=np.float64)
        real = torch.float32 if _dt(dtype) == 1 else torch.float64
        self.device = torch.device(device)
        self.psi = torch.empty(self.batch * (2 << self.n), dtype=real, device=self.device)
        self.lam = torch.empty_like(self.psi)
        self.static_workspace = bool(static_workspace)
        self.work = None
        if not self.static_workspace:
            L = _declare()
            self.work = torch.empty(int(L.qvm_adjoint_workspace_bytes(self.n, self.batch, self.gates.n)),
                                    dtype=torch.uint8, device=self.device)

    def group_count(self):
        """Gate groups of the sweep: one pass over the batch each, forward
        and in reverse."""
        out = ctypes.c_int32()
        check(_declare().qvm_adjoint_group_count(self.n, _dt(self.dtype), self.gates.ptr(), self.gates.n,
                                                 self.pidx.ctypes.data_as(_i32p), self.n_params,
                                                 ctypes.byref(out)))
        return int(out.value)

    def run(self, params, want_grad=True):
        """params: array [batch, n_params].  Returns (f[batch], grad[batch, n_params] or None)."""
        import torch
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(self.batch, self.n_params))
        f = np.zeros(self.batch, dtype=np.float64)
        g = np.zeros((self.batch, self.n_params), dtype=np.float64) if want_grad else None
        stream = torch.cuda.current_stream(self.device).cuda_stream
        common = (self.n, _dt(self.dtype), self.batch, self.gates.ptr(), self.gates.n,
                  self.pidx.ctypes.data_as(_i32p), self.n_params, p.ctypes.data_as(_dp), self.xs.size,
                  self.xs.ctypes.data_as(_u64p), self.zs.ctypes.data_as(_u64p), self.cs.ctypes.data_as(_dp),
                  self.psi.data_ptr(), self.lam.data_ptr())
        outs = (f.ctypes.data_as(_dp), g.ctypes.data_as(_dp) if want_grad else None)
        L = _declare()
        with torch.cuda.device(self.device):
            if self.static_workspace:
                check(L.qvm_adjoint_expect_grad_static(*common, stream, *outs))
            else:
                check(L.qvm_adjoint_expect_grad(*common, self.work.data_ptr(), self.work.numel(), stream, *outs))
        return f, g


_FN = None


def _function():
    global _FN
    if _FN is not None:
        return _FN
    import torch

    class AdjointExpectation(torch.autograd.Function):
        """f = <psi(theta)|H|psi(theta)> per row of theta [batch, n_params];
        the gradient comes from the same reverse-sweep call as f."""

        @staticmethod
        def forward(ctx, theta, problem):
            f, g = problem.run(theta.detach().cpu().numpy(), want_grad=theta.requires_grad)
            if g is not None:
                ctx.save_for_backward(torch.from_numpy(g).to(theta.device, theta.dtype))
            return torch.from_numpy(f).to(theta.device, theta.dtype)

        @staticmethod
        def backward(ctx, grad_f):
            (g,) = ctx.saved_tensors
            return grad_f[:, None] * g, None

    _FN = AdjointExpectation
    return _FN


def adjoint_expectation(theta, problem):
    """Differentiable batched expectation (torch tensors in and out)."""
    return _function().apply(theta, problem)
