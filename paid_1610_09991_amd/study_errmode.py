"""Global against per-integral error control on the same machinery.

For one container (transfer momentum l, particle-hole channel) and a sweep
of the flow scale Omega, integrate all form-factor pairs twice: with the
global criterion of Sec. 3 / Alg. 2 (the summed error of all pairs against
rtol times the summed values) and with every pair held to its own tolerance
(the semantics of integrating each pair separately).  MaxTask of Listing 2
is fixed: batch = batch_max = B leaves per round.  Reports integrand
evaluations, leaves, rounds and time per Omega, and how far the two answers
are apart in units of rtol.

    python -m paid_1610_09991_amd.study_errmode --out study.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = (  # (l, form-factor box order, MaxTask B)
    ((1.57, 1.31), 1, 10),
    ((2.88, 0.26), 1, 10),
    ((1.57, 1.31), 2, 7),
    ((2.88, 0.26), 2, 7),
)


def run(omegas, rtol=1e-6, params=(1.0, -0.25, -0.95, 0.01), log=print):
    sys.path.insert(0, os.path.dirname(HERE))
    import torch  # noqa: F401  (one HIP runtime)
    import paid_1610_09991_amd as P
    import workloads as W

    t, tp, mu, T = params
    rows = []
    for l, L, B in CASES:
        ff = W.ff_box(L)
        M = ff.shape[0]
        ctxs = {
            "global": P.Context(err_mode=P.ERR_GLOBAL, batch=B, batch_max=B, max_regions=1 << 20,
                                max_active=1),
            "per_integral": P.Context(err_mode=P.ERR_PER_INTEGRAL, batch=B, batch_max=B,
                                      max_regions=1 << 20, max_active=1),
        }
        for om in omegas:
            row = {"l": l, "integrals": M * (M + 1) // 2, "B": B, "Omega": om}
            vals = {}
            for name, ctx in ctxs.items():
                out, _, st, rc = ctx.integrate([(t, tp, mu, T, om)], [l], ff, L, P.PH, rtol=rtol)
                vals[name] = out.reshape(M, M)
                row[name] = {"kernel_evals": st["kernel_evals"], "regions": st["regions"],
                             "rounds": st["launch_rounds"], "seconds": st["seconds"],
                             "converged": rc == 0}
            g, p = vals["global"], vals["per_integral"]
            scale = np.maximum(np.abs(p), 1e-3 * np.abs(p).max())
            row["max_diff_in_rtol"] = float(np.max(np.abs(g - p) / scale) / rtol)
            rows.append(row)
            log(f"l=({l[0]:.2f},{l[1]:.2f}) M={M:2d} B={B:2d} Omega={om:8.4f}: evals global "
                f"{row['global']['kernel_evals']:.3e} per-integral {row['per_integral']['kernel_evals']:.3e} "
                f"(x{row['per_integral']['kernel_evals'] / row['global']['kernel_evals']:.2f}); time "
                f"{row['global']['seconds']:.3f} / {row['per_integral']['seconds']:.3f} s; "
                f"|global - per| <= {row['max_diff_in_rtol']:.2f} rtol")
        for c in ctxs.values():
            c.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--points", type=int, default=7)
    a = ap.parse_args(argv)
    omegas = list(10.0 ** np.linspace(1.0, -2.0, a.points))
    rows = run(omegas)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
