"""Write tests/golden/hard_refs.npz: oracle values for the hardest corners of
the workloads (the lowest flow scales of the 20-scale workload, T = 0.005 at
Omega = 0.01 with 9 and 25 form factors, the random batched rows without a
clamp on T or Omega, sampled rows of the 64-set workload).

Calls only the CPU oracle (oracle/) and the seeded input generators
(workloads/).  The oracle runs at rtol 1e-10 (a ten-thousandth of the parity
tests' rtol 1e-6) with the global criterion of Sec. 3 / Alg. 2 and MaxTask 4,
and each stored value comes with the oracle's own per-pair error estimate
(sum over leaves of |Q_N - Q_2N|).  Takes about 40 minutes on 8 cores:

    python tests/golden/make_hard_refs.py [--threads 8]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

RTOL = 1e-10
OUT = os.path.join(HERE, "hard_refs.npz")


def cases():
    """name -> (params [n][5], q [n][2], channel [n], L, ff)"""
    out = {}
    rng = np.random.default_rng(2024)
    # the 20-scale workload at its three lowest scales (Omega 0.0215, 0.0147,
    # 0.01): q at the van Hove momenta (-pi, 0) and (0, -pi), q = 0 and one
    # seeded grid point, both channels
    c2 = W.config("C2")
    qi = [12, 288, 300, int(rng.integers(0, 576))]
    rows = []
    for ip in (17, 18, 19):
        for iq in qi:
            for ch in (O.PP, O.PH):
                rows.append((c2["params"][ip], c2["q"][iq], ch))
    out["c2_low"] = rows
    # T = 0.005 at Omega = 0.01 (the 25-form-factor workload's parameters):
    # q = (-pi, 0) and seeded grid points of the 32 x 32 grid
    c4 = W.config("C4")
    q4 = c4["q"]
    for name, nq in (("c4_ff9", 3), ("c4_ff25", 2)):
        picks = [16] + [int(i) for i in rng.choice(len(q4), nq - 1, replace=False)]
        out[name] = [(c4["params"][0], q4[i], ch) for i in picks for ch in (O.PP, O.PH)]
    # random batched rows without a clamp on T or Omega (T 0.007..0.045,
    # Omega 0.01..0.89), two q of the 16 x 16 grid each
    p6 = W.random_params(6, seed=3, omega_range=(0.01, 1.0))
    q16 = W.q_grid(16)
    out["batched_unclamped"] = [(p6[i], q16[iq], ch) for i in range(6) for iq in (17, 100)
                                for ch in (O.PP, O.PH)]
    # the 64-set workload: its lowest-T row, its lowest-Omega row and two
    # seeded rows, one seeded q each
    c3 = W.config("C3")
    P3 = c3["params"]
    r3 = [int(P3[:, 3].argmin()), int(P3[:, 4].argmin())] + \
        [int(i) for i in rng.choice(len(P3), 2, replace=False)]
    out["c3_sample"] = [(P3[i], c3["q"][int(rng.integers(0, len(c3["q"])))], ch)
                        for i in r3 for ch in (O.PP, O.PH)]
    ffs = {"c2_low": 1, "c4_ff9": 1, "c4_ff25": 2, "batched_unclamped": 1, "c3_sample": 1}
    return {k: (v, ffs[k]) for k, v in out.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    O.build(force=False)
    data = {}
    for name, (rows, L) in cases().items():
        ff = W.ff_box(L)
        conts = [O.Container(ff, L, t=p[0], tp=p[1], mu=p[2], T=p[3], Omega=p[4], lx=q[0],
                             ly=q[1], channel=ch) for p, q, ch in rows]
        t0 = time.perf_counter()
        vals, errs, sts, nc = O.integrate_batch(conts, rtol=RTOL, err_mode=O.ERR_GLOBAL, batch=4,
                                                nthreads=args.threads)
        assert nc == 0, (name, nc)
        print(f"{name}: {len(rows)} containers, {time.perf_counter() - t0:.0f} s, "
              f"{sum(s['regions'] for s in sts)} leaves", flush=True)
        data[f"{name}/params"] = np.array([r[0] for r in rows])
        data[f"{name}/q"] = np.array([r[1] for r in rows])
        data[f"{name}/channel"] = np.array([r[2] for r in rows], dtype=np.int32)
        data[f"{name}/L"] = np.array(L)
        data[f"{name}/value"] = vals
        data[f"{name}/err"] = errs
    data["rtol"] = np.array(RTOL)
    np.savez_compressed(OUT, **data)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
