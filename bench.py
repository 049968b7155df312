#!/usr/bin/env python3
"""Throughput of the adaptive Brillouin-zone quadrature on one MI355X.

One step = one call of the library over the whole realistic workload: t=1,
t'=-0.25, mu=-0.95 (near van Hove), T=0.01, 20 flow scales log-spaced from 10
to 0.01, 24x24 transfer momenta, 9 form factors, both channels, rtol 1e-6:
23,040 containers, 1,036,800 integrals.  Inputs are synthetic (seeded, see
workloads/), outputs stay in device memory.

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (region evaluation, timed with HIP events on its launch stream inside
the library) and the oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "integrals/s at rtol 1e-6, plain vs batched+learned-seeded, 1 MI355X"
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64: vector (256 CUs x 4 SIMD x 16 lanes x 2 x 2.4 GHz) and matrix

# Algorithmic work of one region-evaluation work item (a parent and its four
# children, rule pair N = 4 / 2N = 8, shared 17 x 17 node grid), in FP64 flops
# (an FMA counts 2):
#   integrand: 289 nodes x 80 (dispersion 12, close-pair switch 8, interval
#              arguments 4, two Horner chains of degree 13 = 52, combine 4);
#              a node needs two chains (two values, or one value and its
#              divided difference); the third chain that the branch-free
#              evaluation computes and discards is not counted;
#   separable projection with NP = NB(NB+1)/2 axis products, NB = 2L+1:
#     y-sums  2 x 17 x NP x 27 (fine: 9 mul + 9 FMA) + 2 x 9 x NP x 10 (coarse: 5 FMA)
#     x-sums  4 children x NP^2 x 42 (fine 9 x (mul + FMA), coarse 5 x (mul + FMA))
#     pairs   4 children x MB(MB+1)/2 x 3
#   dense projection (matrix cores): 4 children x 2 M^2 (81 + 25).
K_FLOPS_PER_NODE = 80

# HBM bytes per work item of the region-evaluation kernel, from the
# FETCH_SIZE / WRITE_SIZE counters scaled by a plain copy's readings
# (profiles/k_children_c2_counters.md); valid only for the kernel they were
# taken with, identified by this hash of the two files that define it.
TRAFFIC_BYTES_PER_ITEM = 2416
TRAFFIC_SOURCES_SHA256 = "ed6ac3d5f5a8c23fb8f124b476fbb5c2c1dfaff29bf849d92444f958632854f9"


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paid_1610_09991_amd", "csrc")
    for f in ("paid_device.h", "region_eval.hip"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()
NODES_PER_ITEM = 289


def item_flops(M: int, L: int, separable: bool) -> int:
    k = NODES_PER_ITEM * K_FLOPS_PER_NODE
    if not separable:
        return k + 4 * 2 * M * M * (81 + 25)
    nb = 2 * L + 1
    np_ = nb * (nb + 1) // 2
    mb = nb * nb
    return (k + 2 * 17 * np_ * 27 + 2 * 9 * np_ * 10 + 4 * np_ * np_ * 42
            + 4 * mb * (mb + 1) // 2 * 3)


def computed_pairs(ff, L: int) -> int:
    """Form-factor pairs (m <= n) the half-zone mode computes: all but those
    of two form factors of definite and opposite parity under p -> -p (a box
    function is odd when it has one sine factor), which vanish by symmetry."""
    nb = 2 * L + 1
    odd = [((a // nb > 0 and (a // nb) % 2 == 0) != (a % nb > 0 and (a % nb) % 2 == 0))
           for a in range(nb * nb)]
    par = []
    for row in np.asarray(ff):
        ps = {odd[a] for a in range(nb * nb) if row[a] != 0.0}
        par.append(ps.pop() if len(ps) == 1 else None)
    M = len(par)
    return sum(1 for i in range(M) for j in range(i, M)
               if par[i] is None or par[j] is None or par[i] == par[j])


def cpu_baseline(cfg, budget_s: float, threads: int, seed: int = 11):
    """The oracle as it stands on a seeded sample of the same workload:
    every flow scale, `nq` random transfer momenta of the grid, both channels."""
    import oracle as O
    import workloads as W
    rng = np.random.default_rng(seed)
    nq = 4
    qi = rng.choice(len(cfg["q"]), size=nq, replace=False)
    conts = []
    for p in cfg["params"]:
        for i in qi:
            for ch in (O.PP, O.PH):
                conts.append(O.Container(cfg["ff"], cfg["L"], t=p[0], tp=p[1], mu=p[2], T=p[3],
                                         Omega=p[4], lx=cfg["q"][i][0], ly=cfg["q"][i][1],
                                         channel=ch))
    M = cfg["ff"].shape[0]
    t0 = time.perf_counter()
    _, _, sts, nc = O.integrate_batch(conts, rtol=cfg["rtol"], err_mode=O.ERR_GLOBAL, batch=1,
                                      nthreads=threads)
    dt = time.perf_counter() - t0
    n_int = len(conts) * M * (M + 1) // 2
    return {"value": n_int / dt, "unit": "integrals/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(conts)} containers of the same workload (all 20 scales x {nq} "
                      f"seeded q x 2 channels), serial Alg. 2 per container, OpenMP over "
                      f"containers, {dt:.1f} s wall, budget {budget_s:.0f} s",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--variants", action="store_true", help="also time one call per flow scale")
    ap.add_argument("--gram", choices=["separable", "mfma"], default="separable")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3"], default="fp64",
                    help="arithmetic of the matrix-core projection (with --gram mfma)")
    ap.add_argument("--seed-model", default=None,
                    help="model file of the learned seeding (default: the shipped one)")
    ap.add_argument("--no-seed", action="store_true", help="time the plain batched scheme only")
    ap.add_argument("--no-half-zone", action="store_true",
                    help="skip the extra variant that integrates the half zone p_y >= 0 (an "
                         "exact symmetry of the integrand, not the paper's scheme; never the "
                         "headline value)")
    ap.add_argument("--tuned", default=None,
                    help="autotuner profile (JSON) whose config to apply; default: the shipped "
                         "profile of the workload if there is one")
    ap.add_argument("--graph", type=int, default=1, help="replay each round as a HIP graph")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="with a reduced precision: integrate the workload once more in FP64 and "
                         "report the deviation of every integral in units of the gate")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (the reference "
                         "for scaling the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the containers would shard across GPUs with no exchange during integration",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": n * 8}))
        return
    import paid_1610_09991_amd as P
    import workloads as W

    cfg = W.config(args.workload)
    params, q, ff, L = cfg["params"], cfg["q"], cfg["ff"], cfg["L"]
    M = ff.shape[0]
    MU = M * (M + 1) // 2
    nch = 2
    n_ctr = len(params) * len(q) * nch
    n_int = n_ctr * MU
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    prec = {"fp64": P.FP64, "fp32": P.FP32, "bf16x3": P.BF16X3}[args.precision]
    tuned = {}
    tpath = args.tuned or os.path.join(ROOT, "paid_1610_09991_amd", f"tuned_{args.workload.lower()}.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tuned = json.load(f)["config"]
    ctx = P.Context(stream=stream.cuda_stream, profile=1, precision=prec, graph=args.graph,
                    gram=P.GRAM_SEPARABLE if args.gram == "separable" else P.GRAM_MFMA, **tuned)
    out = torch.empty((len(params), len(q), nch, M, M), dtype=torch.float64, device=dev)
    run = lambda o, c=ctx: c.integrate(params, q, ff, L, P.PP | P.PH, rtol=cfg["rtol"], out=o)

    # learned seeding: the shipped model (trained on the library's own trees,
    # see paid_1610_09991_amd/seed_model.py) with its tuned threshold
    from paid_1610_09991_amd import seed_model as SM
    model = None
    mpath = args.seed_model or SM.DEFAULT_MODEL
    if not args.no_seed and os.path.exists(mpath):
        w_seed, meta = SM.load(mpath)
        model = {"file": os.path.relpath(mpath, ROOT), "kappa": meta["kappa"],
                 "trees": meta["trees"], "train_seconds": meta["train_seconds"],
                 "mse_held_out": meta["mse_held_out"]}

    def timed(seeded, tag, c=ctx, run=run):
        if seeded:
            c.set_seed_model(w_seed, kappa=model["kappa"])
        else:
            c.set_seed_model(None)
        for i in range(args.warmup):
            _, _, st, rc = run(out, c)
            print(f"# {tag} warmup {i}: {st['seconds']:.3f} s, regions {st['regions']}, "
                  f"evals {st['kernel_evals']:.4g}, rc {rc}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = []
        for i in range(args.steps):
            _, _, st, rc = run(out, c)
            sts.append(st)
            print(f"# {tag} step {i}: {st['seconds']:.3f} s, regions {st['regions']}, "
                  f"evals {st['kernel_evals']:.4g}, rc {rc}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, sts

    variants = {}
    dt_plain, st_plain = timed(False, "batched")
    variants["batched"] = {"value": n_int * args.steps / dt_plain,
                           "ms_per_step": 1e3 * dt_plain / args.steps,
                           "kernel_evals": st_plain[-1]["kernel_evals"],
                           "regions": st_plain[-1]["regions"]}
    head, dt, stats = "batched", dt_plain, st_plain
    if model is not None:
        dt_seed, st_seed = timed(True, "batched+learned")
        variants["batched_learned"] = {"value": n_int * args.steps / dt_seed,
                                       "ms_per_step": 1e3 * dt_seed / args.steps,
                                       "kernel_evals": st_seed[-1]["kernel_evals"],
                                       "regions": st_seed[-1]["regions"],
                                       "seed_seconds": st_seed[-1]["seed_seconds"]}
        head, dt, stats = "batched_learned", dt_seed, st_seed
    if not args.no_half_zone:
        # the same integrals from the half zone p_y >= 0 (the integrand is even
        # under p -> -p): an extra data point beside the paper's full-zone scheme
        hctx = P.Context(stream=stream.cuda_stream, profile=1, precision=prec, graph=args.graph,
                         gram=P.GRAM_SEPARABLE if args.gram == "separable" else P.GRAM_MFMA,
                         symmetry=1, **tuned)
        hout = torch.empty_like(out)
        run_h = lambda o, c: c.integrate(params, q, ff, L, P.PP | P.PH, rtol=cfg["rtol"], out=hout)
        dt_half, st_half = timed(False, "batched+half-zone", hctx, run_h)
        hctx.close()
        # only the integrals computed count: the pairs of odd joint parity
        # are zero by the symmetry, not computed, and are left out
        n_even = n_ctr * computed_pairs(ff, L)
        variants["batched_half_zone"] = {"value": n_even * args.steps / dt_half,
                                         "unit": "integrals/s (pairs of even parity only)",
                                         "integrals_per_step": n_even,
                                         "ms_per_step": 1e3 * dt_half / args.steps,
                                         "kernel_evals": st_half[-1]["kernel_evals"],
                                         "regions": st_half[-1]["regions"]}
    ms = 1e3 * dt / args.steps
    value = n_int * args.steps / dt

    items = sum(s["eval_items"] for s in stats)
    ev_s = sum(s["eval_seconds"] for s in stats)
    launches = sum(s["eval_launches"] for s in stats)
    sep = ctx.cfg.gram == P.GRAM_SEPARABLE
    fpi = item_flops(M, L, sep)
    flops_launch = fpi * items / max(launches, 1)
    avg_launch = ev_s / max(launches, 1)
    achieved = flops_launch / avg_launch / 1e12 if avg_launch > 0 else 0.0
    traffic = None
    if sep and M == 9 and kernel_sources_sha256() == TRAFFIC_SOURCES_SHA256:
        traffic = TRAFFIC_BYTES_PER_ITEM * items / max(launches, 1)
    roof = {"bound": "alu" if sep else "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
            "traffic_unit": "B per launch",
            "kernel": "k_children (region evaluation, %s projection)" %
                      ("separable FP64" if sep else "FP64 matrix-core"),
            "launches": launches, "avg_launch_ms": 1e3 * avg_launch, "flops_per_item": fpi,
            "items": items, "eval_share_of_step": ev_s / dt}

    line = {"metric": METRIC, "value": value, "unit": "integrals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if args.precision == "fp64" else f"{args.precision} projection, f64 sums",
            "data": "synthetic",
            "config": {"workload": f"{cfg['name']}: {cfg['desc']}", "containers": n_ctr,
                       "integrals_per_step": n_int,
                       "variant": {"batched": "batched (all containers in one call)",
                                   "batched_learned": "batched, learned seeding"}[head],
                       "err_mode": "global", "rule": "Clenshaw-Curtis N=4/2N=8",
                       "launch": {"graph": args.graph, **(tuned or {"batch": 8, "batch_max": 1024})},
                       "regions_per_step": stats[-1]["regions"],
                       "splits_per_step": stats[-1]["splits"]},
            "roofline": roof, "variants": variants}
    if model is not None:
        line["seed_model"] = model

    if args.compare_fp64 and args.precision != "fp64":
        red = out.cpu().numpy()
        ref_ctx = P.Context(stream=stream.cuda_stream, graph=args.graph, **tuned)
        ref = torch.empty_like(out)
        ref_ctx.integrate(params, q, ff, L, P.PP | P.PH, rtol=cfg["rtol"], out=ref)
        torch.cuda.synchronize()
        r = ref.cpu().numpy().reshape(-1, M, M)
        d = np.abs(red.reshape(-1, M, M) - r)
        scale = np.maximum(np.abs(r), 1e-3 * np.abs(r).max(axis=(1, 2), keepdims=True))
        g = (d / (cfg["rtol"] * scale)).ravel()
        line["error_vs_fp64"] = {"integrals": int(g.size), "gate_units_max": float(g.max()),
                                 "gate_units_median": float(np.median(g)),
                                 "gate_units_p999": float(np.quantile(g, 0.999)),
                                 "note": "|x - x_fp64| / (rtol max(|x_fp64|, 1e-3 max|x_fp64| of "
                                         "the container)) over every integral"}
        ref_ctx.close()

    if args.variants:
        ctx.set_seed_model(None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for p in params:  # plain: one call per flow scale
            ctx.integrate(p[None, :], q, ff, L, P.PP | P.PH, rtol=cfg["rtol"])
        torch.cuda.synchronize()
        variants["plain_per_scale"] = {"value": n_int / (time.perf_counter() - t1)}

    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget, threads)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
