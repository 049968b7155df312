#!/usr/bin/env python3
"""Throughput of the adaptive Brillouin-zone quadrature on one MI355X.

Headline (one step = one call of the library over the whole workload): the
20-scale workload, t=1, t'=-0.25, mu=-0.95 (near van Hove), T=0.01, 20 flow
scales log-spaced from 10 to 0.01, 24x24 transfer momenta, 9 form factors,
both channels, rtol 1e-6: 23,040 containers, 1,036,800 integrals, batched in
one call with learned seeding, the global error criterion of Sec. 3 / Alg. 2.
Inputs are synthetic (seeded, see workloads/), outputs stay in device memory.

Beside the headline, the same JSON line carries (each with one warm-up call
and min(steps, 3) timed calls):
  - the other variants of the metric on the same workload: plain (one call per
    flow scale), batched without seeding, and batched with every integral held
    to its own tolerance (per-integral error control);
  - the 64-set workload (32,768 containers, one call) and the held-out rows of
    the learned seeding (18,432 containers), plain and seeded, each with its
    own roofline entry and CPU-oracle rate.
Every call must converge (status PAID_OK, no container at its region budget);
a call that does not makes the benchmark fail.

Also printed: a roofline entry for the dominant kernel (region evaluation,
timed with HIP events on its launch stream inside the library), the oracle
timed on a bounded sample on the host cores, and the worst deviation of the
headline's integrals at the three lowest scales from the stored oracle values
(tests/golden/hard_refs.npz) in units of the parity gate.
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
#   integrand: 289 nodes x 72 (dispersion 4, close-pair switch 8, interval
#              arguments 4, two Horner chains of degree 13 = 52, combine 4),
#              plus 17 node columns x 8: along a column the two energies
#              are affine in the row's cosine, -2t (cx + cy) - 4t' cx cy - mu
#              = (-2t cx - mu) + cy (-2t - 4t' cx), i.e. 2 FMAs per column
#              and energy and one FMA per node and energy; a node needs two
#              chains (two values, or one value and its divided
#              difference); the third chain that the branch-free evaluation
#              computes and discards is not counted;
#   separable projection with NP = NB(NB+1)/2 axis products, NB = 2L+1:
#     y-sums  2 x 17 x NP x 27 (fine: 9 mul + 9 FMA) + 2 x 9 x NP x 10 (coarse: 5 FMA)
#     x-sums  4 children x NP^2 x 42 (fine 9 x (mul + FMA), coarse 5 x (mul + FMA))
#     pairs   4 children x MB(MB+1)/2 x 3
#   dense projection (matrix cores): 4 children x 2 M^2 (81 + 25).
# This is the method's work in the cheapest form of each step the library
# uses (the separable projection, the per-column energies); work an
# implementation adds (shared edge nodes evaluated once per child: 324 node
# evaluations instead of 289) is not counted.
K_FLOPS_PER_NODE = 72
COLUMNS_PER_ITEM = 17
K_FLOPS_PER_COLUMN = 8

# HBM bytes per work item of the region-evaluation kernel, from the
# FETCH_SIZE / WRITE_SIZE counters scaled by a plain copy's readings
# (profiles/k_children_c2_counters.md); valid only for the kernel they were
# taken with, identified by this hash of the two files that define it.
TRAFFIC_BYTES_PER_ITEM = 2471
TRAFFIC_SOURCES_SHA256 = "72f43a61f2f7d824f78660c0e192a3f483e22e6bb9ae10837f50923c3a6f2734"
NODES_PER_ITEM = 289

# Per-workload region budget (max_regions): the smallest power of two that
# every container of the workload converges within.  The pool holds
# W = pool bytes / (budget x record) containers at once, so a budget just
# large enough admits the most containers per round (C2: 2^17 against 2^18
# gives the same trees, 3,200 instead of 1,600 resident containers and -6%
# per call; C5 likewise -9%).  A container that reaches its budget stops
# with PAID_ENOCONV, which makes the benchmark fail.
BUDGET = {"C2": 1 << 17, "C3": 1 << 19, "C5": 1 << 17, "C2_per_integral": 1 << 19}
# Two kinds of pool slots (paid_config.small_regions / big_share) where they
# pay: C3's containers start in slots of 2^17 leaves and the few that outgrow
# them move to slots of 2^19 (a quarter of the pool): 2,785 resident
# containers instead of 858 and the same trees (-11% per call).  On C2 and in
# the per-integral mode more resident containers were slower.
POOL = {"C3": {"small_regions": 1 << 17, "big_share": 0.25}}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paid_1610_09991_amd", "csrc")
    for f in ("paid_device.h", "region_eval.hip"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def item_flops(M: int, L: int, separable: bool) -> int:
    k = NODES_PER_ITEM * K_FLOPS_PER_NODE + COLUMNS_PER_ITEM * K_FLOPS_PER_COLUMN
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


def cpu_baseline(cfg, budget_s: float, threads: int, seed: int = 11, nq: int = 4,
                 max_rows: int | None = None):
    """The oracle as it stands on a seeded sample of the same workload: every
    parameter row (or `max_rows` seeded rows), `nq` random transfer momenta of
    the grid, both channels."""
    import oracle as O
    rng = np.random.default_rng(seed)
    qi = rng.choice(len(cfg["q"]), size=nq, replace=False)
    rows = np.arange(len(cfg["params"]))
    if max_rows is not None and max_rows < len(rows):
        rows = np.sort(rng.choice(rows, size=max_rows, replace=False))
    conts = []
    for ip in rows:
        p = cfg["params"][ip]
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
    # the serial algorithm on one core: every 16th container of the same sample
    one = conts[::16]
    t1 = time.perf_counter()
    O.integrate_batch(one, rtol=cfg["rtol"], err_mode=O.ERR_GLOBAL, batch=1, nthreads=1)
    d1 = time.perf_counter() - t1
    return {"value": n_int / dt, "unit": "integrals/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(conts)} containers of the same workload ({len(rows)} parameter rows "
                      f"x {nq} seeded q x 2 channels), serial Alg. 2 per container, OpenMP over "
                      f"containers, {dt:.1f} s wall, budget {budget_s:.0f} s",
            "seconds": dt, "host_cpu": host_cpu(),
            "single_thread": {"value": len(one) * M * (M + 1) // 2 / d1, "unit": "integrals/s",
                              "cores": 1, "sample": f"every 16th container of the sample "
                                                    f"({len(one)}), {d1:.1f} s"}}


def host_cpu() -> str:
    """Model name of the host processor (from /proc/cpuinfo) and its thread count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name}, {os.cpu_count()} threads visible"


class Runner:
    """One library context and output buffer for one workload."""

    def __init__(self, P, torch, cfg, stream, tuned, err_mode, max_regions, args, pool=None):
        self.P, self.torch, self.cfg = P, torch, cfg
        prec = {"fp64": P.FP64, "fp32": P.FP32, "bf16x3": P.BF16X3}[args.precision]
        kw = dict(tuned)
        if max_regions:
            kw["max_regions"] = max_regions
        if pool:
            kw.update(pool)
        self.ctx = P.Context(stream=stream.cuda_stream, profile=1, precision=prec,
                             graph=args.graph, eval_layout=args.eval_layout,
                             gram=P.GRAM_SEPARABLE if args.gram == "separable" else P.GRAM_MFMA,
                             err_mode=err_mode, **kw)
        M = cfg["ff"].shape[0]
        self.M = M
        self.n_ctr = len(cfg["params"]) * len(cfg["q"]) * 2
        self.n_int = self.n_ctr * M * (M + 1) // 2
        self.out = torch.empty((len(cfg["params"]), len(cfg["q"]), 2, M, M), dtype=torch.float64,
                               device="cuda:0")

    def call(self, params=None):
        P, cfg = self.P, self.cfg
        p = cfg["params"] if params is None else params
        out = self.out if params is None else None
        _, _, st, rc = self.ctx.integrate(p, cfg["q"], cfg["ff"], cfg["L"], P.PP | P.PH,
                                          rtol=cfg["rtol"], out=out)
        if rc != P.OK or st["not_converged"] != 0:
            raise RuntimeError(f"{cfg['name']}: status {rc}, {st['not_converged']} containers "
                               "at their region budget: not a converged rate")
        return st

    def one_step(self, per_scale: bool):
        """one step: the whole workload in one call, or one call per parameter row"""
        if not per_scale:
            return [self.call()]
        return [self.call(self.cfg["params"][i:i + 1]) for i in range(len(self.cfg["params"]))]

    def timed(self, tag, warmup, steps, model=None, kappa=None, per_scale=False):
        if model is not None:
            self.ctx.set_seed_model(model, kappa=kappa)
        else:
            self.ctx.set_seed_model(None)
        for i in range(warmup):
            sts = self.one_step(per_scale)
            print(f"# {tag} warmup {i}: {sum(s['seconds'] for s in sts):.3f} s, regions "
                  f"{sum(s['regions'] for s in sts)}", file=sys.stderr, flush=True)
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, ends = [], []
        for i in range(steps):
            sts = self.one_step(per_scale)  # each call returns after its stream is idle
            ends.append(time.perf_counter())
            stats += sts
            print(f"# {tag} step {i}: {sum(s['seconds'] for s in sts):.3f} s, regions "
                  f"{sum(s['regions'] for s in sts)}, evals {sum(s['kernel_evals'] for s in sts):.4g}",
                  file=sys.stderr, flush=True)
        self.torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        per_step = len(stats) // steps
        last = stats[-per_step:]
        step_s = np.diff(np.array([t0] + ends))
        return {"value": self.n_int * steps / dt, "ms_per_step": 1e3 * dt / steps,
                "median_ms_per_step": float(1e3 * np.median(step_s)),
                "steps": steps, "warmup": warmup,
                "regions": sum(s["regions"] for s in last),
                "kernel_evals": sum(s["kernel_evals"] for s in last),
                "launch_rounds": sum(s["launch_rounds"] for s in last),
                "seed_seconds": sum(s["seed_seconds"] for s in last)}, stats, dt

    def roofline(self, stats, dt):
        P = self.P
        items = sum(s["eval_items"] for s in stats)
        ev_s = sum(s["eval_seconds"] for s in stats)
        launches = sum(s["eval_launches"] for s in stats)
        sep = self.ctx.cfg.gram == P.GRAM_SEPARABLE
        fpi = item_flops(self.M, self.cfg["L"], sep)
        flops_launch = fpi * items / max(launches, 1)
        avg_launch = ev_s / max(launches, 1)
        achieved = flops_launch / avg_launch / 1e12 if avg_launch > 0 else 0.0
        traffic = None
        if sep and self.M == 9 and kernel_sources_sha256() == TRAFFIC_SOURCES_SHA256:
            traffic = TRAFFIC_BYTES_PER_ITEM * items / max(launches, 1)
        return {"bound": "alu" if sep else "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                "traffic_unit": "B per launch",
                "kernel": "k_children (region evaluation, %s projection)" %
                          ("separable FP64" if sep else "FP64 matrix-core"),
                "launches": launches, "avg_launch_ms": 1e3 * avg_launch, "flops_per_item": fpi,
                "items": items, "eval_share_of_step": ev_s / dt}

    def close(self):
        self.ctx.close()


def golden_check(out, cfg):
    """worst |gpu - oracle| over the stored oracle values of the three lowest
    scales, in units of the gate rtol max(|ref|, 1e-3 max|ref|)"""
    path = os.path.join(ROOT, "tests", "golden", "hard_refs.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    o = out.cpu().numpy()
    worst, n = 0.0, 0
    for k in range(len(z["c2_low/value"])):
        ip = int(np.where(np.all(cfg["params"] == z["c2_low/params"][k], axis=1))[0][0])
        iq = int(np.where(np.all(cfg["q"] == z["c2_low/q"][k], axis=1))[0][0])
        ref = z["c2_low/value"][k]
        g = o[ip, iq, int(z["c2_low/channel"][k])]
        sc = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        worst = max(worst, float((np.abs(g - ref) / (cfg["rtol"] * sc)).max()))
        n += 1
    return {"containers": n, "worst_gate_ratio": worst,
            "reference": "oracle at rtol 1e-10 (tests/golden/hard_refs.npz), scales 0.0215, "
                         "0.0147, 0.01, q at (-pi,0), (0,-pi), 0 and one seeded point"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--quick", action="store_true",
                    help="headline only (no other variants or workloads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--gram", choices=["separable", "mfma"], default="separable")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3"], default="fp64",
                    help="arithmetic of the matrix-core projection (with --gram mfma)")
    ap.add_argument("--seed-model", default=None,
                    help="model file of the learned seeding (default: the shipped one)")
    ap.add_argument("--no-seed", action="store_true", help="time the plain batched scheme only")
    ap.add_argument("--half-zone", action="store_true",
                    help="also time the half-zone mode (p_y >= 0 with the parity of the pairs; "
                         "an exact symmetry of the integrand, not the paper's scheme)")
    ap.add_argument("--tuned", default=None,
                    help="autotuner profile (JSON) whose config to apply; default: the shipped "
                         "profile")
    ap.add_argument("--graph", type=int, default=1, help="replay each round as a HIP graph")
    ap.add_argument("--eval-layout", type=int, default=0,
                    help="region-evaluation kernel: 0 the fastest for the basis, 1 one wave "
                         "per parent")
    ap.add_argument("--err-mode", choices=["global", "per_integral"], default="global")
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
    from paid_1610_09991_amd import seed_model as SM

    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    tpath = args.tuned or os.path.join(ROOT, "paid_1610_09991_amd", "tuned_c2.json")
    with open(tpath) as f:
        tuned = json.load(f)["config"]
    model = None
    mpath = args.seed_model or SM.DEFAULT_MODEL
    if not args.no_seed and os.path.exists(mpath):
        w_seed, meta = SM.load(mpath)
        model = {"file": os.path.relpath(mpath, ROOT), "kappa": meta["kappa"],
                 "trees": meta["trees"], "train_seconds": meta["train_seconds"],
                 "mse_held_out": meta["mse_held_out"]}
    em_head = P.ERR_GLOBAL if args.err_mode == "global" else P.ERR_PER_INTEGRAL
    threads = min(16, os.cpu_count() or 1)

    # ---------------------------------------------------------------- headline
    cfg = W.config(args.workload)
    budget = BUDGET.get(args.workload if args.err_mode == "global"
                        else args.workload + "_per_integral", 1 << 20)
    run = Runner(P, torch, cfg, stream, tuned, em_head, budget, args,
                 POOL.get(args.workload) if args.err_mode == "global" else None)
    variants = {}
    res, st_b, dt_b = run.timed("batched", args.warmup if model is None else min(args.warmup, 1),
                                args.steps if model is None else min(args.steps, 3))
    variants["batched"] = res
    head, stats, dt = "batched", st_b, dt_b
    if model is not None:
        res, st_s, dt_s = run.timed("batched+learned", args.warmup, args.steps, w_seed,
                                    model["kappa"])
        variants["batched_learned"] = res
        head, stats, dt = "batched_learned", st_s, dt_s
    line_parity = golden_check(run.out, cfg) if args.workload == "C2" else None
    roof = run.roofline(stats, dt)
    hv = variants[head]
    M = run.M
    line = {"metric": METRIC, "value": hv["value"], "unit": "integrals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": hv["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if args.precision == "fp64" else f"{args.precision} projection, f64 sums",
            "data": "synthetic",
            "config": {"workload": f"{cfg['name']}: {cfg['desc']}", "containers": run.n_ctr,
                       "integrals_per_step": run.n_int,
                       "variant": {"batched": "batched (all containers in one call)",
                                   "batched_learned": "batched, learned seeding"}[head],
                       "err_mode": args.err_mode, "rule": "Clenshaw-Curtis N=4/2N=8",
                       "launch": {"graph": args.graph, "eval_layout": args.eval_layout,
                                  "max_regions": budget, **tuned,
                                  **(POOL.get(args.workload, {}) if args.err_mode == "global" else {})},
                       "regions_per_step": hv["regions"]},
            "roofline": roof, "variants": variants}
    if line_parity is not None:
        line["parity_vs_oracle"] = line_parity
    if model is not None:
        line["seed_model"] = model

    if args.compare_fp64 and args.precision != "fp64":
        red = run.out.cpu().numpy()
        ref_ctx = P.Context(stream=stream.cuda_stream, graph=args.graph, max_regions=budget, **tuned)
        ref = torch.empty_like(run.out)
        ref_ctx.integrate(cfg["params"], cfg["q"], cfg["ff"], cfg["L"], P.PP | P.PH,
                          rtol=cfg["rtol"], out=ref)
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

    sec_steps = min(args.steps, 3)
    if not args.quick and args.workload == "C2" and args.err_mode == "global":
        # plain: one call per flow scale, the scales one after another
        res, _, _ = run.timed("plain per scale", 1, sec_steps, per_scale=True)
        variants["plain_per_scale"] = res
        if args.half_zone:
            hrun = Runner(P, torch, cfg, stream, dict(tuned, symmetry=1), P.ERR_GLOBAL, budget,
                          args)
            res, _, _ = hrun.timed("batched+half-zone", 1, sec_steps)
            n_even = run.n_ctr * computed_pairs(cfg["ff"], cfg["L"])
            res["value"] *= n_even / run.n_int
            res["unit"] = "integrals/s (pairs of even parity only)"
            variants["batched_half_zone"] = res
            hrun.close()
    run.close()
    if not args.quick and args.workload == "C2" and args.err_mode == "global":
        # every integral held to its own tolerance (the survey's metric runs)
        prun = Runner(P, torch, cfg, stream, tuned, P.ERR_PER_INTEGRAL,
                      BUDGET["C2_per_integral"], args)
        res, _, _ = prun.timed("batched per-integral", 1, sec_steps)
        res["err_mode"] = "per_integral"
        variants["batched_per_integral"] = res
        prun.close()
        # the other workloads of the metric, each in one call per step
        others = {}
        for wl in ("C3", "C5"):
            wcfg = W.config(wl)
            wrun = Runner(P, torch, wcfg, stream, tuned, P.ERR_GLOBAL, BUDGET[wl], args, POOL.get(wl))
            entry = {"workload": f"{wcfg['name']}: {wcfg['desc']}", "containers": wrun.n_ctr,
                     "integrals_per_step": wrun.n_int, "max_regions": BUDGET[wl],
                     "pool": POOL.get(wl, {}), "variants": {}}
            res, st, dtw = wrun.timed(f"{wl} batched", 1, sec_steps)
            entry["variants"]["batched"] = res
            if model is not None:
                res, st, dtw = wrun.timed(f"{wl} batched+learned", 1, sec_steps, w_seed,
                                          model["kappa"])
                entry["variants"]["batched_learned"] = res
            entry["roofline"] = wrun.roofline(st, dtw)
            wrun.close()
            if not args.no_cpu_baseline:
                entry["cpu_baseline"] = cpu_baseline(wcfg, 10.0, threads, nq=2, max_rows=8)
            others[wl] = entry
        line["workloads"] = others

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget, threads)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
