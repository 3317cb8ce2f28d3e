"""Python handle on the learned Davidson preconditioner (argument
marshalling over the C ABI; forward, backward, Adam and training run in the
HIP library)."""
import ctypes

import numpy as np

from . import binding as B


def _torch():
    import torch
    return torch


class MLP:
    def __init__(self, width=256, seed=0):
        self.lib = B.load()
        h = ctypes.c_void_p()
        B.check(self.lib.dmrg_mlp_create(width, seed, ctypes.byref(h)), self.lib)
        self.handle = h
        self.width = width
        self.n_params = int(self.lib.dmrg_mlp_num_params(h))

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        B.check(self.lib.dmrg_mlp_get_params(self.handle, out.ctypes.data, self.n_params), self.lib)
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        B.check(self.lib.dmrg_mlp_set_params(self.handle, p.ctypes.data, p.size), self.lib)

    @staticmethod
    def _stream(stream):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    @staticmethod
    def _dev(t):
        torch = _torch()
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    def forward(self, x, stream=None):
        torch = _torch()
        x = x.contiguous()
        g = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        B.check(self.lib.dmrg_mlp_forward(self.handle, self._dev(x), x.shape[0], self._dev(g),
                                          self._stream(stream)), self.lib)
        return g

    def step(self, diag, r, seg_off, theta, sigma, rnorm, floor=1e-2, stream=None):
        """Learned correction t (CUDA float64) of one preconditioning step
        for the segments seg_off (host) with per-segment theta, sigma and
        residual norms (host sequences), as dmrg_davidson computes it."""
        import numpy as np
        torch = _torch()
        assert diag.dtype == torch.float64 and r.dtype == torch.float64 and diag.is_cuda and r.is_cuda
        diag, r = diag.contiguous(), r.contiguous()
        t = torch.empty_like(r)
        off = np.ascontiguousarray(seg_off, dtype=np.int64)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        sg = np.ascontiguousarray(sigma, dtype=np.float64)
        rn = np.ascontiguousarray(rnorm, dtype=np.float64)
        B.check(self.lib.dmrg_mlp_step(self.handle, ctypes.c_void_p(diag.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                       len(th), off.ctypes.data, th.ctypes.data, sg.ctypes.data, rn.ctypes.data,
                                       floor, ctypes.c_void_p(t.data_ptr()), self._stream(stream)), self.lib)
        return t

    def loss_grad(self, x, a, b, stream=None):
        torch = _torch()
        x, a, b = x.contiguous(), a.contiguous(), b.contiguous()
        gr = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = ctypes.c_double()
        B.check(self.lib.dmrg_mlp_loss_grad(self.handle, self._dev(x), self._dev(a), self._dev(b),
                                            x.shape[0], ctypes.byref(loss), self._dev(gr),
                                            self._stream(stream)), self.lib)
        return loss.value, gr

    def adam_step(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        B.check(self.lib.dmrg_mlp_adam_step(self.handle, self._dev(grad.contiguous()), lr, beta1,
                                            beta2, eps, self._stream(stream)), self.lib)

    def train(self, x, a, b, steps=2000, batch=4096, lr=1e-3, seed=1, beta1=0.9, beta2=0.999,
              eps=1e-8, trace=False, stream=None):
        """Minibatch Adam; returns the per-step loss trace (numpy) if asked."""
        x, a, b = x.contiguous(), a.contiguous(), b.contiguous()
        o = B.TrainOpts(lr, beta1, beta2, eps, batch, steps, seed)
        tr = np.zeros(steps, dtype=np.float32) if trace else None
        B.check(self.lib.dmrg_mlp_train(self.handle, self._dev(x), self._dev(a), self._dev(b),
                                        x.shape[0], ctypes.byref(o),
                                        tr.ctypes.data if trace else None, self._stream(stream)),
                self.lib)
        return tr

    def free(self):
        if getattr(self, "handle", None):
            self.lib.dmrg_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
