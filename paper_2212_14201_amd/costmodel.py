"""The cost-model MLP on the library's HIP kernels (binding of qvm_mlp_*).

Parameters, Adam moments and activations live in torch device tensors; every
forward, backward and update step runs in libqvm.  ``save``/``load`` keep the
weights and the optimiser state so that training can resume.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .qvm import check, lib

_fp = ctypes.c_void_p


def _declare():
    L = lib()
    L.qvm_mlp_param_count.argtypes = [ctypes.c_int, ctypes.c_int]
    L.qvm_mlp_param_count.restype = ctypes.c_size_t
    L.qvm_mlp_forward.argtypes = [ctypes.c_int] * 3 + [_fp] * 4 + [_fp]
    L.qvm_mlp_forward.restype = ctypes.c_int
    L.qvm_mlp_backward.argtypes = [ctypes.c_int] * 3 + [_fp] * 8 + [_fp]
    L.qvm_mlp_backward.restype = ctypes.c_int
    L.qvm_mlp_adam_step.argtypes = [ctypes.c_size_t, _fp, _fp, _fp, _fp, ctypes.c_int,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _fp]
    L.qvm_mlp_adam_step.restype = ctypes.c_int
    return L


class CostMLP:
    def __init__(self, d, hidden=128, init=None, device="cuda"):
        import torch
        L = _declare()
        self.d, self.h = int(d), int(hidden)
        self.device = torch.device(device)
        self.count = int(L.qvm_mlp_param_count(self.d, self.h))
        self.params = torch.zeros(self.count, dtype=torch.float32, device=self.device)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        if init is not None:
            self.set_params(init)

    # packed <-> list of arrays [W1, b1, W2, b2, W3, b3]
    def set_params(self, arrays):
        import torch
        flat = np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrays])
        assert flat.size == self.count
        self.params.copy_(torch.from_numpy(flat.astype(np.float32)))

    def unpack(self, flat):
        d, h = self.d, self.h
        sizes = [d * h, h, h * h, h, h, 1]
        shapes = [(d, h), (h,), (h, h), (h,), (h, 1), (1,)]
        out, o = [], 0
        for s, sh in zip(sizes, shapes):
            out.append(flat[o:o + s].reshape(sh))
            o += s
        return out

    def get_params(self):
        return self.unpack(self.params.cpu().numpy().astype(np.float64))

    def get_grads(self):
        return self.unpack(self.grads.cpu().numpy().astype(np.float64))

    def _stream(self):
        import torch
        return torch.cuda.current_stream(self.device).cuda_stream

    def forward(self, X):
        """X: torch float32 [B, d] on the device.  Returns (y [B], act)."""
        import torch
        B = X.shape[0]
        act = torch.empty(4 * B * self.h, dtype=torch.float32, device=self.device)
        y = torch.empty(B, dtype=torch.float32, device=self.device)
        check(_declare().qvm_mlp_forward(B, self.d, self.h, X.data_ptr(), self.params.data_ptr(),
                                         act.data_ptr(), y.data_ptr(), self._stream()))
        return y, act

    def backward(self, X, t, act, y):
        """Fills self.grads with dL/dparams; returns the loss tensor [1]."""
        import torch
        B = X.shape[0]
        work = torch.empty(2 * B * self.h + B, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check(_declare().qvm_mlp_backward(B, self.d, self.h, X.data_ptr(), t.data_ptr(),
                                          self.params.data_ptr(), act.data_ptr(), y.data_ptr(),
                                          self.grads.data_ptr(), work.data_ptr(), loss.data_ptr(),
                                          self._stream()))
        return loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        check(_declare().qvm_mlp_adam_step(self.count, self.params.data_ptr(), self.grads.data_ptr(),
                                           self.m.data_ptr(), self.v.data_ptr(), self.step, lr,
                                           beta1, beta2, eps, self._stream()))

    def train_step(self, X, t, lr):
        y, act = self.forward(X)
        loss = self.backward(X, t, act, y)
        self.adam(lr)
        return loss

    def predict(self, X):
        y, _ = self.forward(X)
        return y

    def save(self, path, extra=None):
        np.savez(path, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(), step=self.step, d=self.d, h=self.h,
                 **(extra or {}))

    @classmethod
    def load(cls, path, device="cuda"):
        import torch
        z = np.load(path, allow_pickle=False)
        net = cls(int(z["d"]), int(z["h"]), device=device)
        net.params.copy_(torch.from_numpy(z["params"]))
        net.m.copy_(torch.from_numpy(z["m"]))
        net.v.copy_(torch.from_numpy(z["v"]))
        net.step = int(z["step"])
        return net, z
