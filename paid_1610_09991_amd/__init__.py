"""Python binding of libpaid: the MI355X (gfx950) adaptive Brillouin-zone
quadrature of the scale-derivative bubbles of the truncated-unity fRG
(arXiv:1610.09991).

This module only marshals arguments into the C ABI declared in
``include/paid.h``; every step of the computation runs in the library's HIP
kernels.  PyTorch tensors are accepted for device-resident outputs and a
torch stream may be handed to the library; nothing else of torch is used.
If ``libpaid.so`` has not been built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaid.so")

OK, ENOCONV, EINVAL, ENOMEM, EDEVICE, EINTERNAL = 0, 1, -1, -2, -3, -4
BUBBLE_DOT, BUBBLE, UNIT, GAUSS = 0, 1, 2, 3
PP, PH = 1, 2
ERR_GLOBAL, ERR_PER_INTEGRAL = 0, 1
FP64, FP32, BF16X3 = 0, 1, 2
GRAM_MFMA, GRAM_SEPARABLE = 0, 1


class PaidError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpaid error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("device", C.c_int), ("N", C.c_int), ("batch", C.c_int), ("batch_max", C.c_int),
                ("err_mode", C.c_int), ("precision", C.c_int), ("gram", C.c_int),
                ("kind", C.c_int), ("nu", C.c_double), ("max_regions", C.c_long),
                ("max_active", C.c_int), ("pool_gib", C.c_double),
                ("gauss", C.c_double * 3), ("stream", C.c_void_p), ("profile", C.c_int)]


class Params(C.Structure):
    _fields_ = [("t", C.c_double), ("tp", C.c_double), ("mu", C.c_double),
                ("T", C.c_double), ("Omega", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("containers", C.c_long), ("not_converged", C.c_long), ("regions", C.c_long),
                ("splits", C.c_long), ("kernel_evals", C.c_long), ("rounds", C.c_long),
                ("launch_rounds", C.c_long), ("max_depth", C.c_int), ("max_active", C.c_int),
                ("seconds", C.c_double), ("eval_seconds", C.c_double), ("eval_launches", C.c_long),
                ("eval_items", C.c_long)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ("paid_config_default", "paid_create", "paid_integrate", "paid_kernel_eval",
           "paid_children_eval", "paid_destroy", "paid_last_error")

_lib = None


def lib():
    """Load libpaid.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paid_1610_09991_amd/build.py "
                               "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.paid_config_default.argtypes = [C.POINTER(Config)]
        L.paid_create.argtypes = [C.POINTER(vp), C.POINTER(Config)]
        L.paid_integrate.argtypes = [vp, vp, C.c_int, vp, C.c_int, vp, C.c_int, C.c_int,
                                     C.c_uint, C.c_double, C.c_double, vp, vp, C.POINTER(Stats)]
        L.paid_kernel_eval.argtypes = [vp, vp, C.c_uint, vp, vp, C.c_int, vp]
        L.paid_children_eval.argtypes = [vp, vp, vp, C.c_uint, vp, C.c_int, C.c_int, vp, C.c_int,
                                         vp, vp]
        L.paid_destroy.argtypes = [vp]
        L.paid_last_error.argtypes = [vp]
        L.paid_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(a):
    """Address of a numpy array or a torch tensor (host or device)."""
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def params_array(rows) -> np.ndarray:
    """Rows (t, t', mu, T, Omega) as a contiguous [n][5] float64 array."""
    return _f64(rows).reshape(-1, 5)


class Context:
    """A libpaid context (device workspace, tables, stream)."""

    def __init__(self, device=0, stream=None, **cfg):
        L = lib()
        c = Config()
        L.paid_config_default(C.byref(c))
        c.device = device
        for k, v in cfg.items():
            if k == "gauss":
                for i in range(3):
                    c.gauss[i] = float(v[i])
            elif not hasattr(c, k):
                raise TypeError(f"unknown config field {k}")
            else:
                setattr(c, k, v)
        if stream is not None:
            c.stream = stream if isinstance(stream, int) else getattr(stream, "cuda_stream", stream)
        self.cfg = c
        h = C.c_void_p()
        rc = L.paid_create(C.byref(h), C.byref(c))
        if rc != OK:
            raise PaidError(rc, L.paid_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().paid_destroy(self.h)
            self.h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, allow_noconv=True):
        if rc == OK or (rc == ENOCONV and allow_noconv):
            return rc
        raise PaidError(rc, lib().paid_last_error(self.h).decode())

    def integrate(self, params, q, ff, ff_L, channels=PP | PH, rtol=1e-6, atol=0.0, out=None,
                  err=False):
        """All containers (parameter row, q, channel).  Returns (out, err_out,
        stats, status); out is [n_params][n_q][n_ch][M][M].  `out` may be a
        preallocated torch tensor (device) or numpy array."""
        p = params_array(params)
        qa = _f64(q).reshape(-1, 2)
        ffa = _f64(ff)
        M = ffa.shape[0]
        nch = (1 if channels & PP else 0) + (1 if channels & PH else 0)
        shape = (p.shape[0], qa.shape[0], nch, M, M)
        if out is None:
            out = np.zeros(shape)
        e = np.zeros(shape) if err is True else (err if err is not False else None)
        st = Stats()
        rc = lib().paid_integrate(self.h, _ptr(p), p.shape[0], _ptr(qa), qa.shape[0], _ptr(ffa),
                                  M, ff_L, channels, rtol, atol, _ptr(out),
                                  _ptr(e) if e is not None else None, C.byref(st))
        self._check(rc)
        return out, e, st.as_dict(), rc

    def kernel(self, param_row, a, b, channel=PH):
        p = params_array([param_row])
        a = _f64(a).ravel()
        b = _f64(b).ravel()
        out = np.zeros_like(a)
        self._check(lib().paid_kernel_eval(self.h, _ptr(p), channel, _ptr(a), _ptr(b), a.size,
                                           _ptr(out)), allow_noconv=False)
        return out

    def children(self, param_row, l, channel, ff, ff_L, codes):
        """Q_2N and keys of the four children of each parent code (d, ix, iy)."""
        p = params_array([param_row])
        la = _f64(l).ravel()
        ffa = _f64(ff)
        M = ffa.shape[0]
        cd = np.ascontiguousarray(codes, dtype=np.int32).reshape(-1, 3)
        n = cd.shape[0]
        q2n = np.zeros((n, 4, M * (M + 1) // 2))
        er = np.zeros((n, 4))
        self._check(lib().paid_children_eval(self.h, _ptr(p), _ptr(la), channel, _ptr(ffa), M,
                                             ff_L, _ptr(cd), n, _ptr(q2n), _ptr(er)),
                    allow_noconv=False)
        return q2n, er
