"""ctypes binding of the surrogate C ABI (include/surrogate.h); argument marshalling only."""
import ctypes as C
import os
import re

import numpy as np

from . import rve

HEADER = os.path.join(os.path.dirname(rve.HERE), "include", "surrogate.h")

NPARAM = 33664
BF16, BF16X3 = 0, 1


class SurrogateDesc(C.Structure):
    _fields_ = [("A0", C.c_double * 16), ("c_scale", C.c_double * 3), ("w_scale", C.c_double),
                ("seed", C.c_uint64)]


class TrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("lr_final", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("wP", C.c_float),
                ("wA", C.c_float), ("rhoP", C.c_float), ("rhoA", C.c_float), ("seed", C.c_uint64),
                ("precision", C.c_int32)]


_done = False


def lib():
    global _done
    L = rve.lib()
    if not _done:
        vp, i32, i64, dp, fp = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
        L.rve_train_opts_default.argtypes = [C.POINTER(TrainOpts)]
        L.rve_train_opts_default.restype = None
        L.rve_surrogate_create.argtypes = [C.POINTER(SurrogateDesc), C.POINTER(vp)]
        L.rve_surrogate_destroy.argtypes = [vp]
        L.rve_surrogate_set_params.argtypes = [vp, vp]
        L.rve_surrogate_get_params.argtypes = [vp, vp]
        L.rve_surrogate_eval.argtypes = [vp, vp, vp, vp, vp, i64, i32, vp]
        L.rve_surrogate_loss_grad.argtypes = [vp, vp, vp, vp, i64, C.POINTER(TrainOpts), vp, C.POINTER(dp), vp]
        L.rve_surrogate_adam_step.argtypes = [vp, vp, C.POINTER(TrainOpts), vp]
        L.rve_surrogate_train.argtypes = [vp, vp, vp, vp, i64, C.POINTER(TrainOpts), vp, vp]
        L.rve_surrogate_calibrate.argtypes = [vp, vp, vp, i64, i32, vp]
        L.rve_surrogate_select.argtypes = [vp, i64, fp, vp, vp, vp]
        _done = True
    return L


def declared_functions():
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void)\s+(rve_\w+)\s*\(", txt, flags=re.M)))


def train_opts(**kw):
    o = TrainOpts()
    lib().rve_train_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _p(t):
    return rve._ptr(t)


def _s(stream):
    return C.c_void_p(stream) if stream is not None else None


class Surrogate:
    """rve_surrogate handle.  Device tensors: F, P [n,4] float64, A [n,16] float64,
    indicator [n] float32, gradients [NPARAM] float32."""

    def __init__(self, A0, c_scale=(0.5, 0.5, 0.5), w_scale=0.1, seed=1):
        d = SurrogateDesc((C.c_double * 16)(*[float(v) for v in np.asarray(A0, np.float64).reshape(16)]),
                          (C.c_double * 3)(*[float(v) for v in c_scale]), float(w_scale), int(seed))
        h = C.c_void_p()
        rve.check(lib().rve_surrogate_create(C.byref(d), C.byref(h)), "rve_surrogate_create")
        self.h = h

    @staticmethod
    def _dev(t, numel, dtype, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous() \
                or t.numel() != numel:
            raise ValueError(f"{name}: expected a contiguous {dtype} GPU tensor with {numel} elements")

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, np.float32)
        if th.size != NPARAM:
            raise ValueError("theta has the wrong size")
        rve.check(lib().rve_surrogate_set_params(self.h, _p(th)), "rve_surrogate_set_params")

    def get_params(self):
        th = np.zeros(NPARAM, np.float32)
        rve.check(lib().rve_surrogate_get_params(self.h, _p(th)), "rve_surrogate_get_params")
        return th

    def eval(self, F, P, A=None, indicator=None, precision=BF16X3, stream=None):
        import torch
        n = F.numel() // 4
        self._dev(F, 4 * n, torch.float64, "F")
        self._dev(P, 4 * n, torch.float64, "P")
        if A is not None:
            self._dev(A, 16 * n, torch.float64, "A")
        if indicator is not None:
            self._dev(indicator, n, torch.float32, "indicator")
        rve.check(lib().rve_surrogate_eval(self.h, _p(F), _p(P), _p(A), _p(indicator), n, precision, _s(stream)),
                  "rve_surrogate_eval")

    def loss_grad(self, F, P, A, opts=None, stream=None):
        import torch
        n = F.numel() // 4
        self._dev(F, 4 * n, torch.float64, "F")
        self._dev(P, 4 * n, torch.float64, "P")
        self._dev(A, 16 * n, torch.float64, "A")
        g = torch.empty(NPARAM, dtype=torch.float32, device=F.device)
        L = C.c_double()
        o = opts if opts is not None else train_opts()
        rve.check(lib().rve_surrogate_loss_grad(self.h, _p(F), _p(P), _p(A), n, C.byref(o), _p(g), C.byref(L),
                                                _s(stream)), "rve_surrogate_loss_grad")
        return L.value, g

    def adam_step(self, grad, opts=None, stream=None):
        import torch
        self._dev(grad, NPARAM, torch.float32, "grad")
        o = opts if opts is not None else train_opts()
        rve.check(lib().rve_surrogate_adam_step(self.h, _p(grad), C.byref(o), _s(stream)), "rve_surrogate_adam_step")

    def train(self, F, P, A, opts=None, stream=None):
        import torch
        n = F.numel() // 4
        self._dev(F, 4 * n, torch.float64, "F")
        self._dev(P, 4 * n, torch.float64, "P")
        self._dev(A, 16 * n, torch.float64, "A")
        o = opts if opts is not None else train_opts()
        loss = np.zeros(max(o.steps, 1), np.float32)
        rve.check(lib().rve_surrogate_train(self.h, _p(F), _p(P), _p(A), n, C.byref(o), _p(loss), _s(stream)),
                  "rve_surrogate_train")
        return loss[:o.steps]

    def calibrate(self, F, P, precision=BF16X3, stream=None):
        import torch
        n = F.numel() // 4
        self._dev(F, 4 * n, torch.float64, "F")
        self._dev(P, 4 * n, torch.float64, "P")
        rve.check(lib().rve_surrogate_calibrate(self.h, _p(F), _p(P), n, precision, _s(stream)),
                  "rve_surrogate_calibrate")

    def destroy(self):
        if self.h is not None:
            rve.check(lib().rve_surrogate_destroy(self.h), "rve_surrogate_destroy")
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def select(indicator, threshold, stream=None):
    """Device int32 list of the indices whose indicator exceeds threshold, and its
    device count."""
    import torch
    n = indicator.numel()
    idx = torch.empty(max(n, 1), dtype=torch.int32, device=indicator.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=indicator.device)
    rve.check(lib().rve_surrogate_select(_p(indicator), n, float(threshold), _p(idx), _p(cnt), _s(stream)),
              "rve_surrogate_select")
    return idx, cnt
