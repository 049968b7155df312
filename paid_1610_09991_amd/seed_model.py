"""The learned seeding's model: training data from the library's own trees,
GPU training, a sweep of the seed threshold, and the model file.

Everything here drives the C ABI (paid_integrate with label output,
paid_seed_train, paid_mlp_forward); no arithmetic of the method or the model
runs in Python.  Run as a module to rebuild the shipped model file:

    python -m paid_1610_09991_amd.seed_model --out paid_1610_09991_amd/seed_c5.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "seed_c5.npz")


def generate(ctx, calls, ff, L, rtol=1e-6):
    """Features [n][7] and labels [n][256] of the converged plain trees of
    every container of every (params, q) call."""
    import paid_1610_09991_amd as P
    xs, ys, t0, nreg = [], [], time.perf_counter(), 0
    ctx.set_seed_model(None)
    for prm, q in calls:
        n = len(prm) * len(q) * 2
        f = np.zeros((n, 7), dtype=np.float32)
        y = np.zeros((n, 256), dtype=np.float32)
        ctx.set_label_output(f, y)
        _, _, st, _ = ctx.integrate(prm, q, ff, L, P.PP | P.PH, rtol=rtol)
        nreg += st["regions"]
        xs.append(f)
        ys.append(y)
    ctx.set_label_output(None, None)
    return np.concatenate(xs), np.concatenate(ys), time.perf_counter() - t0, nreg


def train(ctx, x, y, steps=6000, batch=256, lr=2e-3, lr_final=5e-5, seed=1):
    t0 = time.perf_counter()
    w, hist = ctx.seed_train(x, y, steps=steps, batch=batch, lr=lr, lr_final=lr_final, seed=seed)
    return w, hist, time.perf_counter() - t0


def mse(ctx, w, x, y):
    yh = ctx.mlp_forward(w, x)
    return float(np.mean((yh.astype(np.float64) - y) ** 2))


def sweep_kappa(ctx, w, prm, q, ff, L, kappas=(0.5, 1.0, 2.0, 4.0), rtol=1e-6, repeat=2):
    """Integrate held-out rows without seeding and with each threshold
    4 kappa; returns per variant the evaluations, leaves and best time."""
    import paid_1610_09991_amd as P
    res = {}
    variants = [("plain", None)] + [(f"kappa={k:g}", k) for k in kappas]
    for name, k in variants:
        ctx.set_seed_model(None if k is None else w, kappa=k or 1.0)
        best = None
        for _ in range(repeat):
            _, _, st, rc = ctx.integrate(prm, q, ff, L, P.PP | P.PH, rtol=rtol)
            best = st if best is None or st["seconds"] < best["seconds"] else best
        res[name] = {"kernel_evals": best["kernel_evals"], "regions": best["regions"],
                     "seconds": best["seconds"], "rounds": best["launch_rounds"]}
    ctx.set_seed_model(None)
    return res


def save(path, w, meta):
    np.savez(path, w=np.asarray(w, dtype=np.float32), meta=np.array(json.dumps(meta)))


def load(path=DEFAULT_MODEL):
    """(weights float32 [67072], metadata dict); plain arrays only."""
    with np.load(path, allow_pickle=False) as z:
        return z["w"].astype(np.float32), json.loads(str(z["meta"]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--calls", type=int, default=20)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--eval-rows", type=int, default=4, help="held-out rows of the sweep")
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch  # noqa: F401  (one HIP runtime)
    import paid_1610_09991_amd as P
    import workloads as W

    ff, L = W.ff_box(1), 1
    calls = W.c5_training_calls(calls=a.calls)
    ctx = P.Context(max_regions=1 << 18)
    x, y, tgen, nreg = generate(ctx, calls, ff, L)
    print(f"# trees {len(x)} (leaves {nreg}) generated in {tgen:.2f} s", flush=True)
    nval = len(x) // 10  # the last calls are held out
    w, hist, ttr = train(ctx, x[:-nval], y[:-nval], steps=a.steps, batch=a.batch)
    vtr, vval = mse(ctx, w, x[:-nval], y[:-nval]), mse(ctx, w, x[-nval:], y[-nval:])
    base = float(np.mean((y[-nval:] - y[:-nval].mean(axis=0)) ** 2))
    print(f"# trained {a.steps} steps in {ttr:.2f} s: mse train {vtr:.4f} held-out {vval:.4f} "
          f"(mean predictor {base:.4f})", flush=True)
    c5 = W.config("C5")
    prm, q = c5["params"][:a.eval_rows], c5["q"]
    sweep = sweep_kappa(ctx, w, prm, q, ff, L)
    for k, v in sweep.items():
        print(f"# {k:>10}: evals {v['kernel_evals']:.4g} leaves {v['regions']} "
              f"time {v['seconds']:.4f} s rounds {v['rounds']}", flush=True)
    seeded = {k: v for k, v in sweep.items() if k != "plain"}
    best = min(seeded, key=lambda k: seeded[k]["seconds"])
    meta = {"recipe": "c5_training_calls(seed=5, calls=%d, rows=16, nq=32), FF9, rtol 1e-6" % a.calls,
            "trees": int(len(x)), "held_out": int(nval), "steps": a.steps, "batch": a.batch,
            "mse_train": vtr, "mse_held_out": vval, "mse_mean_predictor": base,
            "generate_seconds": tgen, "train_seconds": ttr, "sweep": sweep,
            "kappa": float(best.split("=")[1])}
    save(a.out, w, meta)
    print(json.dumps({"model": a.out, "kappa": meta["kappa"], "mse_held_out": vval}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
