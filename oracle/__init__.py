"""Plain FP64 CPU oracle for the adaptive Brillouin-zone quadrature of the
scale-derivative bubbles (arXiv:1610.09991, Secs. 2-4).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything from here, and the two share no code.

This module is a ctypes shim over ``liboracle.so`` (built from
``paid_oracle.c`` with gcc by :func:`build`).  See ``paid_oracle.h`` for the
definitions each C function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "paid_oracle.c")
# PAID_ORACLE_LIB names another build of the same source (a sanitizer build)
_LIB = os.environ.get("PAID_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

BUBBLE_DOT, BUBBLE, UNIT, GAUSS = 0, 1, 2, 3
PP, PH = 0, 1
MODE_A, MODE_B = 0, 1
ERR_GLOBAL, ERR_PER_INTEGRAL, ERR_WEIGHTED = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O3 for the x86-64-v3 level (AVX2; the
    library built here also runs on the GPU host, so not -march=native),
    -ffp-contract=off so that every product and sum is rounded as written,
    OpenMP only across problems."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Problem(C.Structure):
    _fields_ = [("kind", C.c_int), ("channel", C.c_int),
                ("t", C.c_double), ("tp", C.c_double), ("mu", C.c_double),
                ("T", C.c_double), ("Omega", C.c_double),
                ("lx", C.c_double), ("ly", C.c_double),
                ("ff_L", C.c_int), ("n_ff", C.c_int), ("ff", C.POINTER(C.c_double)),
                ("gx", C.c_double), ("gy", C.c_double), ("gsigma", C.c_double),
                ("pair_w", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("N", C.c_int), ("mode", C.c_int), ("err_mode", C.c_int),
                ("batch", C.c_int), ("rtol", C.c_double), ("atol", C.c_double),
                ("nu", C.c_double), ("max_regions", C.c_long)]


class Stats(C.Structure):
    _fields_ = [("regions", C.c_long), ("splits", C.c_long), ("kernel_evals", C.c_long),
                ("rounds", C.c_long), ("converged", C.c_int), ("max_depth", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.po_cc_rule.argtypes = [C.c_int, dp, dp]
        L.po_hurwitz_zeta.argtypes = [C.c_double, C.c_double]
        L.po_hurwitz_zeta.restype = C.c_double
        L.po_dispersion.argtypes = [C.c_double] * 5
        L.po_dispersion.restype = C.c_double
        L.po_kernel.argtypes = [C.c_int, C.c_int] + [C.c_double] * 4
        L.po_kernel.restype = C.c_double
        L.po_fermi.argtypes = [C.c_double, C.c_double]
        L.po_fermi.restype = C.c_double
        L.po_box_basis.argtypes = [C.c_int, C.c_double, dp]
        L.po_integrand.argtypes = [C.POINTER(Problem), C.c_double, C.c_double]
        L.po_integrand.restype = C.c_double
        L.po_region_eval.argtypes = [C.POINTER(Problem), C.c_int] + [C.c_double] * 4 + [dp, dp]
        L.po_integrate.argtypes = [C.POINTER(Problem), C.POINTER(Options), dp, dp,
                                   C.POINTER(Stats)]
        L.po_integrate_batch.argtypes = [C.POINTER(Problem), C.c_int, C.POINTER(Options),
                                         dp, dp, C.POINTER(Stats), C.c_int]
        L.po_brute.argtypes = [C.POINTER(Problem), C.c_int, dp]
        L.po_mlp_nparams.restype = C.c_long
        L.po_mlp_forward.argtypes = [dp, dp, C.c_int, dp]
        L.po_mlp_loss_grad.argtypes = [dp, dp, dp, C.c_int, dp]
        L.po_mlp_loss_grad.restype = C.c_double
        L.po_mlp_adam.argtypes = [dp, dp, dp, dp, C.c_long, C.c_int, C.c_double]
        ip = C.POINTER(C.c_int)
        L.po_seed_features.argtypes = [C.c_double] * 7 + [C.c_int, dp, ip]
        L.po_tree_labels.argtypes = [dp, C.c_long, dp]
        L.po_integrate_labels.argtypes = [C.POINTER(Problem), C.POINTER(Options), dp, dp,
                                          C.POINTER(Stats), dp]
        L.po_integrate_leaves.argtypes = [C.POINTER(Problem), C.POINTER(Options), dp, dp,
                                          C.POINTER(Stats), dp, dp, C.c_long,
                                          C.POINTER(C.c_long)]
        L.po_seed_tree.argtypes = [dp, C.c_int, C.c_double, C.c_long, dp, ip]
        L.po_seed_tree.restype = C.c_long
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def cc_rule(n: int):
    x = np.zeros(n + 1)
    w = np.zeros(n + 1)
    if lib().po_cc_rule(n, _dp(x), _dp(w)) != 0:
        raise ValueError("bad rule order")
    return x, w


def hurwitz_zeta(s: float, q: float) -> float:
    return lib().po_hurwitz_zeta(float(s), float(q))


def dispersion(t, tp, mu, kx, ky) -> float:
    return lib().po_dispersion(t, tp, mu, kx, ky)


def fermi(e, T) -> float:
    return lib().po_fermi(float(e), float(T))


def kernel(a, b, Omega, T, channel=PH, kind=BUBBLE_DOT) -> float:
    return lib().po_kernel(kind, channel, float(a), float(b), float(Omega), float(T))


def box_basis(L: int, x: float) -> np.ndarray:
    u = np.zeros(2 * L + 1)
    lib().po_box_basis(L, float(x), _dp(u))
    return u


class Container:
    """One adaptive problem: (parameters, scale, transfer momentum, channel)."""

    def __init__(self, ff, ff_L, *, t=1.0, tp=0.0, mu=0.0, T=0.1, Omega=0.1, lx=0.0, ly=0.0,
                 channel=PH, kind=BUBBLE_DOT, gauss=(0.0, 0.0, 1.0), pair_w=None):
        self.ff = np.ascontiguousarray(ff, dtype=np.float64)
        nb = (2 * ff_L + 1) ** 2
        if self.ff.ndim != 2 or self.ff.shape[1] != nb:
            raise ValueError("ff must be [n_ff][(2L+1)^2]")
        self.M = self.ff.shape[0]
        self.pair_w = None if pair_w is None else np.ascontiguousarray(pair_w, dtype=np.float64)
        if self.pair_w is not None and self.pair_w.shape != (self.M, self.M):
            raise ValueError("pair_w must be [n_ff][n_ff]")
        self.s = Problem(kind, channel, t, tp, mu, T, Omega, lx, ly, ff_L, self.M,
                         _dp(self.ff), gauss[0], gauss[1], gauss[2],
                         _dp(self.pair_w) if self.pair_w is not None else None)

    def integrand(self, px, py) -> float:
        return lib().po_integrand(C.byref(self.s), float(px), float(py))

    def region(self, x0, x1, y0, y1, N=4):
        mu = self.M * (self.M + 1) // 2
        qn = np.zeros(mu)
        q2n = np.zeros(mu)
        if lib().po_region_eval(C.byref(self.s), N, x0, x1, y0, y1, _dp(qn), _dp(q2n)) != 0:
            raise ValueError("bad problem")
        return qn, q2n

    def integrate_labels(self, rtol=1e-6, atol=0.0, N=4, err_mode=ERR_GLOBAL, batch=1,
                         nu=1e-3, max_regions=1 << 22):
        """Mode-B integration that also returns the 16x16 labels of the final
        tree (container frame, index 16*j + i)."""
        v = np.zeros((self.M, self.M))
        e = np.zeros((self.M, self.M))
        y = np.zeros(256)
        st = Stats()
        o = Options(N, MODE_B, err_mode, batch, rtol, atol, nu, max_regions)
        rc = lib().po_integrate_labels(C.byref(self.s), C.byref(o), _dp(v), _dp(e), C.byref(st),
                                       _dp(y))
        if rc < 0:
            raise ValueError("bad problem or options")
        return v, e, st.as_dict(), y

    def integrate_leaves(self, rtol=1e-6, atol=0.0, N=4, err_mode=ERR_GLOBAL, batch=1,
                         nu=1e-3, max_regions=1 << 22):
        """Mode-B integration that also returns the final leaves in creation
        order: (value, err, stats, rects [n][4] = (x0, x1, y0, y1), q2n [n][MU])."""
        mu = self.M * (self.M + 1) // 2
        o = Options(N, MODE_B, err_mode, batch, rtol, atol, nu, max_regions)
        v = np.zeros((self.M, self.M))
        e = np.zeros((self.M, self.M))
        st = Stats()
        n = C.c_long(0)
        rc = lib().po_integrate_leaves(C.byref(self.s), C.byref(o), _dp(v), _dp(e), C.byref(st),
                                       None, None, 0, C.byref(n))
        if rc < 0:
            raise ValueError("bad problem or options")
        rects = np.zeros((max(n.value, 1), 4))
        q2n = np.zeros((max(n.value, 1), mu))
        lib().po_integrate_leaves(C.byref(self.s), C.byref(o), _dp(v), _dp(e), C.byref(st),
                                  _dp(rects), _dp(q2n), n.value, C.byref(n))
        return v, e, st.as_dict(), rects[:n.value], q2n[:n.value]

    def brute(self, L: int) -> np.ndarray:
        v = np.zeros((self.M, self.M))
        if lib().po_brute(C.byref(self.s), L, _dp(v)) != 0:
            raise ValueError("bad problem")
        return v

    def integrate(self, rtol=1e-6, atol=0.0, N=4, mode=MODE_B, err_mode=ERR_PER_INTEGRAL,
                  batch=1, nu=1e-3, max_regions=1 << 22):
        v = np.zeros((self.M, self.M))
        e = np.zeros((self.M, self.M))
        st = Stats()
        o = Options(N, mode, err_mode, batch, rtol, atol, nu, max_regions)
        rc = lib().po_integrate(C.byref(self.s), C.byref(o), _dp(v), _dp(e), C.byref(st))
        if rc < 0:
            raise ValueError("bad problem or options")
        return v, e, st.as_dict()


def integrate_batch(containers, rtol=1e-6, atol=0.0, N=4, mode=MODE_B,
                    err_mode=ERR_PER_INTEGRAL, batch=1, nu=1e-3, max_regions=1 << 22,
                    nthreads=1):
    """Integrate many containers (OpenMP over containers when nthreads > 1).

    Returns (values [n][M][M], errs [n][M][M], stats list, n_not_converged)."""
    n = len(containers)
    M = containers[0].M
    if any(c.M != M for c in containers):
        raise ValueError("all containers must share the form-factor count")
    arr = (Problem * n)(*[c.s for c in containers])
    vals = np.zeros((n, M, M))
    errs = np.zeros((n, M, M))
    sts = (Stats * n)()
    o = Options(N, mode, err_mode, batch, rtol, atol, nu, max_regions)
    rc = lib().po_integrate_batch(arr, n, C.byref(o), _dp(vals), _dp(errs), sts, nthreads)
    if rc < 0:
        raise ValueError("bad problem or options")
    return vals, errs, [s.as_dict() for s in sts], rc


# ---------------------------------------------------------------- density model
MLP_IN, MLP_HID, MLP_OUT = 7, 128, 256


def mlp_nparams() -> int:
    return lib().po_mlp_nparams()


def mlp_forward(w, x):
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_IN)
    y = np.zeros((x.shape[0], MLP_OUT))
    lib().po_mlp_forward(_dp(w), _dp(x), x.shape[0], _dp(y))
    return y


def mlp_loss_grad(w, x, y):
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_IN)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1, MLP_OUT)
    g = np.zeros_like(w)
    loss = lib().po_mlp_loss_grad(_dp(w), _dp(x), _dp(y), x.shape[0], _dp(g))
    return loss, g


def mlp_adam(w, g, m, v, t, lr):
    """in place on w, m, v (float64 arrays)"""
    lib().po_mlp_adam(_dp(w), _dp(g), _dp(m), _dp(v), w.size, t, lr)


# ---------------------------------------------------------------- seeding
def seed_features(t, tp, mu, T, Omega, lx, ly, channel):
    """(features[7], cellmap[256]): model inputs and, per container cell,
    the model cell it reads."""
    x = np.zeros(7)
    cm = np.zeros(256, dtype=np.int32)
    lib().po_seed_features(t, tp, mu, T, Omega, lx, ly, channel, _dp(x),
                           cm.ctypes.data_as(C.POINTER(C.c_int)))
    return x, cm


def tree_labels(rects):
    r = np.ascontiguousarray(rects, dtype=np.float64).reshape(-1, 4)
    y = np.zeros(256)
    lib().po_tree_labels(_dp(r), r.shape[0], _dp(y))
    return y


def seed_tree(count, dmax, thresh, limit):
    """(n_leaves, rects [n][4], depth bound used)"""
    cnt = np.ascontiguousarray(count, dtype=np.float64)
    d = C.c_int(0)
    n = lib().po_seed_tree(_dp(cnt), dmax, thresh, limit, None, C.byref(d))
    rects = np.zeros((max(n, 1), 4))
    lib().po_seed_tree(_dp(cnt), dmax, thresh, limit, _dp(rects), C.byref(d))
    return n, rects[:n], d.value


# ---------------------------------------------------------------- contraction
def contract(chi, VP, VC, VD):
    """The contraction beside the integration (Sec. 2, Eqs. matmul-P, matmul-C,
    matmul-D) as written, per transfer momentum, in FP64 with numpy's matrix
    product: chi [n_l][2][M][M] (pp, ph), couplings [n_l][M][M]."""
    chi = np.asarray(chi, dtype=np.float64)
    pp, ph = chi[:, 0], chi[:, 1]
    VP, VC, VD = (np.asarray(a, dtype=np.float64) for a in (VP, VC, VD))
    dP = VP @ pp @ VP
    dC = -(VC @ ph @ VC)
    dD = 2.0 * (VD @ ph @ VD) - VC @ ph @ VD - VD @ ph @ VC
    return dP, dC, dD


def weights_from_couplings(V):
    """Weights of the full matrix entries for which sum_mn |dX_mn| <=
    sum_pq w_pq |d chi_pq| with dX = V chi V: w_pq = (sum_m |V_mp|)(sum_n |V_qn|)."""
    A = np.abs(np.asarray(V, dtype=np.float64))
    return np.outer(A.sum(axis=0), A.sum(axis=1))
