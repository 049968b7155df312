"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Holds no arithmetic of the method: only parameter sets, transfer
momentum grids and form-factor coefficient tables in the documented box-basis
convention, all drawn from ``numpy.random.default_rng(seed)``.

Box basis (per axis): u_0 = 1, u_{2k-1} = sqrt2 cos(k x), u_{2k} = sqrt2 sin(k x)
for k = 1..L; a form factor is sum_{a,b} C[a(2L+1)+b] u_a(p_x) u_b(p_y).

Parameter rows are (t, t', mu, T, Omega).  The workloads mirror the shapes of
the paper's experiments (45 and 325 integrals per transfer momentum, Sec. 5)
on synthetic lattices; the paper's own model parameters are not stated.
"""
from __future__ import annotations

import math

import numpy as np

PP, PH = 0, 1
CH_PP, CH_PH = 1, 2  # channel bit mask used by the library interface


def box_size(L: int) -> int:
    return (2 * L + 1) ** 2


def ff_box(L: int) -> np.ndarray:
    """The full box basis of order L as form factors (identity coefficients)."""
    return np.eye(box_size(L))


def ff5() -> np.ndarray:
    """s, extended-s, d, p_x, p_y (orthonormal), as coefficients over the L=1 box."""
    C = np.zeros((5, 9))
    r = 1.0 / math.sqrt(2.0)
    C[0, 0] = 1.0                       # 1
    C[1, 3] = r; C[1, 1] = r            # cos px + cos py
    C[2, 3] = r; C[2, 1] = -r           # cos px - cos py
    C[3, 6] = 1.0                       # sqrt2 sin px
    C[4, 2] = 1.0                       # sqrt2 sin py
    return C


def q_grid(Lq: int) -> np.ndarray:
    """l_ij = 2 pi (i, j)/Lq with i, j in [-Lq/2, Lq/2)."""
    idx = np.arange(-(Lq // 2), Lq - Lq // 2)
    ii, jj = np.meshgrid(idx, idx, indexing="ij")
    return np.stack([2 * np.pi * ii.ravel() / Lq, 2 * np.pi * jj.ravel() / Lq], axis=1)


def _params(t, tp, mu, T, Om):
    return np.array([[t, tp, mu, T, o] for o in np.atleast_1d(Om)], dtype=np.float64)


def config(name: str, seed: int | None = None) -> dict:
    """Workload dictionaries: params [n][5], q [n_q][2], ff [M][(2L+1)^2], L,
    channels (bit mask), rtol, and a description."""
    if name == "C1":
        return dict(name="C1", params=_params(1.0, 0.0, 0.0, 0.1, 0.1), q=q_grid(8), ff=ff5(),
                    L=1, channels=CH_PP | CH_PH, rtol=1e-4,
                    desc="t=1 t'=0 mu=0 T=0.1 Omega=0.1, 8x8 q, FF5, pp+ph, rtol 1e-4")
    if name == "C2":
        om = 10.0 * 10.0 ** (-3.0 * np.arange(20) / 19.0)
        return dict(name="C2", params=_params(1.0, -0.25, -0.95, 0.01, om), q=q_grid(24),
                    ff=ff_box(1), L=1, channels=CH_PP | CH_PH, rtol=1e-6,
                    desc="t=1 t'=-0.25 mu=-0.95 T=0.01, 20 scales 10..0.01, 24x24 q, FF9, "
                         "pp+ph, rtol 1e-6")
    if name == "C3":
        rng = np.random.default_rng(3 if seed is None else seed)
        n = 64
        mu = rng.uniform(-1.2, 0.0, n)
        T = np.exp(rng.uniform(math.log(0.005), math.log(0.1), n))
        tp = rng.uniform(-0.35, 0.0, n)
        om = np.exp(rng.uniform(math.log(0.01), math.log(1.0), n))
        p = np.stack([np.ones(n), tp, mu, T, om], axis=1)
        return dict(name="C3", params=p, q=q_grid(16), ff=ff_box(1), L=1,
                    channels=CH_PP | CH_PH, rtol=1e-6,
                    desc="64 random sets (seed 3), 16x16 q, FF9, pp+ph, rtol 1e-6")
    if name == "C4":
        return dict(name="C4", params=_params(1.0, -0.3, -1.1, 0.005, [0.01, 0.1]),
                    q=q_grid(32), ff=ff_box(2), L=2, channels=CH_PP | CH_PH, rtol=1e-6,
                    desc="t'=-0.3 mu=-1.1 T=0.005 Omega=0.01,0.1, 32x32 q, FF25, pp+ph")
    if name == "C5":
        rng = np.random.default_rng(6 if seed is None else seed)
        n = 16
        mu = rng.uniform(-1.2, 0.0, n)
        T = np.exp(rng.uniform(math.log(0.005), math.log(0.1), n))
        tp = rng.uniform(-0.35, 0.0, n)
        om = np.exp(rng.uniform(math.log(0.01), math.log(10.0), n))
        p = np.stack([np.ones(n), tp, mu, T, om], axis=1)
        return dict(name="C5", params=p, q=q_grid(24), ff=ff_box(1), L=1,
                    channels=CH_PP | CH_PH, rtol=1e-6,
                    desc="16 held-out random sets (seed 6), 24x24 q, FF9, pp+ph, rtol 1e-6")
    raise KeyError(name)


def c5_training_calls(seed: int = 5, calls: int = 20, rows: int = 16, nq: int = 32):
    """Training set of the learned seeding: per call, `rows` random parameter
    rows of the batched workload's distribution with Omega log-uniform in
    [0.01, 10], and `nq` transfer momenta drawn without replacement from the
    16 x 16 grid; both channels.  The default gives 10,240 trees per channel."""
    rng = np.random.default_rng(seed)
    grid = q_grid(16)
    out = []
    for _ in range(calls):
        mu = rng.uniform(-1.2, 0.0, rows)
        T = np.exp(rng.uniform(math.log(0.005), math.log(0.1), rows))
        tp = rng.uniform(-0.35, 0.0, rows)
        om = np.exp(rng.uniform(math.log(0.01), math.log(10.0), rows))
        p = np.stack([np.ones(rows), tp, mu, T, om], axis=1)
        out.append((p, grid[rng.choice(len(grid), nq, replace=False)]))
    return out


def random_params(n: int, seed: int, omega_range=(0.01, 1.0)) -> np.ndarray:
    """Random parameter rows as in the batched workload."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-1.2, 0.0, n)
    T = np.exp(rng.uniform(math.log(0.005), math.log(0.1), n))
    tp = rng.uniform(-0.35, 0.0, n)
    om = np.exp(rng.uniform(math.log(omega_range[0]), math.log(omega_range[1]), n))
    return np.stack([np.ones(n), tp, mu, T, om], axis=1)


def containers(cfg: dict):
    """Flattened container list in library output order:
    (param index, q index, channel) with channel pp before ph."""
    chans = [c for c, bit in ((PP, CH_PP), (PH, CH_PH)) if cfg["channels"] & bit]
    out = []
    for ip in range(len(cfg["params"])):
        for iq in range(len(cfg["q"])):
            for ch in chans:
                out.append((ip, iq, ch))
    return out
