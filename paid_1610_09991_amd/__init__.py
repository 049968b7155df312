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
ERR_GLOBAL, ERR_PER_INTEGRAL, ERR_WEIGHTED = 0, 1, 2
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
                ("gauss", C.c_double * 3), ("stream", C.c_void_p), ("profile", C.c_int),
                ("graph", C.c_int), ("eval_wg_per_cu", C.c_int), ("symmetry", C.c_int),
                ("eval_layout", C.c_int), ("small_regions", C.c_long), ("big_share", C.c_double)]


class Params(C.Structure):
    _fields_ = [("t", C.c_double), ("tp", C.c_double), ("mu", C.c_double),
                ("T", C.c_double), ("Omega", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("containers", C.c_long), ("not_converged", C.c_long), ("regions", C.c_long),
                ("splits", C.c_long), ("kernel_evals", C.c_long), ("rounds", C.c_long),
                ("launch_rounds", C.c_long), ("max_depth", C.c_int), ("max_active", C.c_int),
                ("seconds", C.c_double), ("eval_seconds", C.c_double), ("eval_launches", C.c_long),
                ("eval_items", C.c_long), ("seeded", C.c_long), ("seed_seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FlowOpts(C.Structure):
    _fields_ = [("omega0", C.c_double), ("omega1", C.c_double), ("rtol", C.c_double),
                ("atol", C.c_double), ("rtol_int", C.c_double), ("h0", C.c_double),
                ("max_steps", C.c_int)]


class FlowStats(C.Structure):
    _fields_ = [("steps", C.c_int), ("rejected", C.c_int), ("evaluations", C.c_int),
                ("kernel_evals", C.c_long), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int), ("batch", C.c_int), ("lr", C.c_float), ("lr_final", C.c_float),
                ("seed", C.c_ulonglong), ("init", C.c_int), ("use_graph", C.c_int)]


MLP_IN, MLP_OUT = 7, 256

EXPORTS = ("paid_config_default", "paid_create", "paid_integrate", "paid_kernel_eval",
           "paid_children_eval", "paid_destroy", "paid_last_error", "paid_mlp_nparams",
           "paid_set_seed_model", "paid_set_label_output", "paid_mlp_forward",
           "paid_mlp_loss_grad", "paid_mlp_adam", "paid_train_opts_default", "paid_seed_train",
           "paid_contract", "paid_flow_opts_default", "paid_flow", "paid_set_pair_weights",
           "paid_mlp_loss_grad_noalloc", "paid_set_leaf_output")

NOALLOC_MAX_N = 2048  # PAID_NOALLOC_MAX_N

_lib = None


def lib():
    """Load libpaid.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paid_1610_09991_amd/build.py "
                               "(or __graft_entry__.build()) first")
        try:
            # torch and libpaid name the same HIP runtime (libamdhip64.so.7);
            # loading torch first makes the process hold one runtime, torch's,
            # so that torch's device memory and streams are valid in libpaid
            import torch  # noqa: F401
        except ImportError:
            pass
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
        L.paid_mlp_nparams.argtypes = []
        L.paid_mlp_nparams.restype = C.c_long
        L.paid_set_seed_model.argtypes = [vp, vp, C.c_int, C.c_double]
        L.paid_set_label_output.argtypes = [vp, vp, vp]
        L.paid_set_pair_weights.argtypes = [vp, vp]
        L.paid_set_leaf_output.argtypes = [vp, vp, vp, C.c_long]
        L.paid_mlp_forward.argtypes = [vp, vp, vp, C.c_int, vp]
        L.paid_mlp_loss_grad.argtypes = [vp, vp, vp, vp, C.c_int, vp, dp]
        L.paid_mlp_loss_grad_noalloc.argtypes = [vp, vp, vp, vp, C.c_int, vp, dp]
        L.paid_mlp_adam.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_float]
        L.paid_train_opts_default.argtypes = [C.POINTER(TrainOpts)]
        L.paid_seed_train.argtypes = [vp, vp, vp, C.c_int, C.POINTER(TrainOpts), vp, vp]
        L.paid_contract.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]
        L.paid_flow_opts_default.argtypes = [C.POINTER(FlowOpts)]
        L.paid_flow.argtypes = [vp, vp, vp, C.c_int, vp, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp,
                                C.POINTER(FlowOpts), C.POINTER(FlowStats)]
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
        if getattr(self, "h", None) and _lib is not None:
            _lib.paid_destroy(self.h)
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

    # ------------------------------------------------------------ learned seeding
    def set_seed_model(self, weights, dmax=8, kappa=2.0):
        """Seed later integrate() calls from this model (None: root start)."""
        if weights is None:
            self._check(lib().paid_set_seed_model(self.h, None, 0, 1.0), allow_noconv=False)
            return
        w = weights if hasattr(weights, "data_ptr") else np.ascontiguousarray(weights, np.float32)
        self._check(lib().paid_set_seed_model(self.h, _ptr(w), dmax, kappa), allow_noconv=False)

    def set_pair_weights(self, w):
        """Pair weights [n_ctr][M][M] of the weighted error mode (kept alive
        here; None clears)."""
        self._pw = None if w is None else (w if hasattr(w, "data_ptr") else _f64(w))
        self._check(lib().paid_set_pair_weights(self.h, _ptr(self._pw) if w is not None else None),
                    allow_noconv=False)

    def set_leaf_output(self, codes=None, q2n=None):
        """Arm the leaf output of later integrate() calls: codes [n_ctr][cap][3]
        int32 and q2n [n_ctr][cap][MU] float64 (kept alive here; None clears)."""
        self._leaves = (codes, q2n)
        cap = 0 if codes is None else codes.shape[1]
        self._check(lib().paid_set_leaf_output(
            self.h, _ptr(codes) if codes is not None else None,
            _ptr(q2n) if q2n is not None else None, cap), allow_noconv=False)

    def set_label_output(self, features=None, labels=None):
        """Arm per-container features [n][7] and tree labels [n][256] (FP32
        arrays or tensors the caller keeps alive) for later integrate() calls."""
        self._lab = (features, labels)
        self._check(lib().paid_set_label_output(
            self.h, _ptr(features) if features is not None else None,
            _ptr(labels) if labels is not None else None), allow_noconv=False)

    def mlp_forward(self, w, x, y=None):
        n = x.shape[0]
        if y is None:
            y = np.zeros((n, MLP_OUT), dtype=np.float32)
        self._check(lib().paid_mlp_forward(self.h, _ptr(w), _ptr(x), n, _ptr(y)),
                    allow_noconv=False)
        return y

    def mlp_loss_grad(self, w, x, y, grad=None):
        n = x.shape[0]
        if grad is None:
            grad = np.zeros(mlp_nparams(), dtype=np.float32)
        loss = C.c_double(0.0)
        self._check(lib().paid_mlp_loss_grad(self.h, _ptr(w), _ptr(x), _ptr(y), n, _ptr(grad),
                                             C.byref(loss)), allow_noconv=False)
        return loss.value, grad

    def mlp_loss_grad_noalloc(self, w, x, y, grad):
        """paid_mlp_loss_grad through the entry point that allocates nothing:
        w, x, y, grad must be device tensors; returns the loss."""
        loss = C.c_double(0.0)
        self._check(lib().paid_mlp_loss_grad_noalloc(self.h, _ptr(w), _ptr(x), _ptr(y), x.shape[0],
                                                     _ptr(grad), C.byref(loss)),
                    allow_noconv=False)
        return loss.value

    def mlp_adam(self, w, g, m, v, t, lr):
        """one Adam step in place on device tensors w, m, v"""
        self._check(lib().paid_mlp_adam(self.h, _ptr(w), _ptr(g), _ptr(m), _ptr(v), t, lr),
                    allow_noconv=False)

    def seed_train(self, x, y, w=None, **opts):
        """Train the density model on the GPU; returns (w, minibatch losses)."""
        o = TrainOpts()
        lib().paid_train_opts_default(C.byref(o))
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown training option {k}")
            setattr(o, k, v)
        if w is None:
            w = np.zeros(mlp_nparams(), dtype=np.float32)
            o.init = 1
        hist = np.zeros(o.steps)
        self._check(lib().paid_seed_train(self.h, _ptr(x), _ptr(y), x.shape[0], C.byref(o), _ptr(w),
                                          _ptr(hist)), allow_noconv=False)
        return w, hist


    # ------------------------------------------------------------ contraction
    def contract(self, chi, VP, VC, VD):
        """dP, dC, dD of Eqs. matmul-P/C/D for chi [n_l][2][M][M] (pp, ph) and
        couplings [n_l][M][M]; numpy in, numpy out (or device tensors)."""
        n_l, M = VP.shape[0], VP.shape[-1]
        if hasattr(VP, "data_ptr"):
            import torch
            outs = [torch.empty_like(VP) for _ in range(3)]
        else:
            chi, VP, VC, VD = (_f64(a) for a in (chi, VP, VC, VD))
            outs = [np.zeros((n_l, M, M)) for _ in range(3)]
        self._check(lib().paid_contract(self.h, n_l, M, _ptr(chi), _ptr(VP), _ptr(VC), _ptr(VD),
                                        *[_ptr(o) for o in outs]), allow_noconv=False)
        return tuple(outs)


    # ------------------------------------------------------------ flow driver
    def flow(self, base, q, ff, ff_L, VP, VC, VD, P0, C0, D0, **opts):
        """Integrate the flow (fixed couplings) from omega0 to omega1; returns
        (P, C, D, stats).  base: (t, t', mu, T)."""
        o = FlowOpts()
        lib().paid_flow_opts_default(C.byref(o))
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown flow option {k}")
            setattr(o, k, v)
        prm = params_array([tuple(base) + (0.0,)])
        qa = _f64(q).reshape(-1, 2)
        ffa = _f64(ff)
        V = [_f64(v) for v in (VP, VC, VD)]
        st = [np.array(_f64(x), copy=True) for x in (P0, C0, D0)]
        fs = FlowStats()
        self._check(lib().paid_flow(self.h, _ptr(prm), _ptr(qa), qa.shape[0], _ptr(ffa),
                                    ffa.shape[0], ff_L, *[_ptr(v) for v in V],
                                    *[_ptr(x) for x in st], C.byref(o), C.byref(fs)),
                    allow_noconv=False)
        return st[0], st[1], st[2], fs.as_dict()


def mlp_nparams() -> int:
    return lib().paid_mlp_nparams()
