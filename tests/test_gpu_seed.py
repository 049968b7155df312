"""GPU tests of the learned seeding against the oracle, through the C ABI:
the density model's forward pass, gradients (FP32 on the GPU against FP64 on
the CPU) and Adam; training with and without a captured HIP graph; the
model features, tree labels and seed trees; integration from a seed tree;
and the gain of a trained model over the plain scheme."""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

NU = 1e-3
THREADS = max(1, min(16, os.cpu_count() or 1))
DIMS = [7, 128, 128, 128, 256]


@pytest.fixture(scope="module")
def P():
    import paid_1610_09991_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def layer_slices():
    out, off = [], 0
    for l in range(4):
        ni, no = DIMS[l], DIMS[l + 1]
        out.append(("W%d" % (l + 1), slice(off, off + no * ni)))
        off += no * ni
        out.append(("b%d" % (l + 1), slice(off, off + no)))
        off += no
    return out


def random_weights(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    w = np.zeros(O.mlp_nparams(), dtype=np.float32)
    for name, sl in layer_slices():
        l = int(name[1]) - 1
        if name[0] == "W":
            w[sl] = rng.normal(0, scale / math.sqrt(DIMS[l]), sl.stop - sl.start)
        else:
            w[sl] = rng.normal(0, 0.1, sl.stop - sl.start)
    return w


def gate_ratio(gpu, ref, rtol):
    scale = np.maximum(np.abs(ref), NU * np.abs(ref).max())
    return float((np.abs(gpu - ref) / (rtol * scale)).max())


# ------------------------------------------------------------------ model kernels
def test_mlp_nparams(P):
    assert P.mlp_nparams() == O.mlp_nparams() == 67072


def test_seed_model_arguments_are_checked(P):
    with P.Context() as c:
        w = np.zeros(P.mlp_nparams(), dtype=np.float32)
        for dmax, kappa in ((13, 2.0), (-1, 2.0), (8, 0.0), (8, float("nan"))):
            with pytest.raises(P.PaidError):
                c.set_seed_model(w, dmax=dmax, kappa=kappa)
        w[5] = np.inf
        with pytest.raises(P.PaidError):
            c.set_seed_model(w)
        c.set_seed_model(None)


@pytest.mark.parametrize("n", [1, 100, 1000])
def test_mlp_forward_matches_oracle(P, n):
    w = random_weights(11)
    x = np.random.default_rng(n).uniform(-1.5, 1.5, (n, 7)).astype(np.float32)
    with P.Context() as c:
        y = c.mlp_forward(w, x)
    ref = O.mlp_forward(w.astype(np.float64), x.astype(np.float64))
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert err <= 1e-5, err


@pytest.mark.parametrize("n", [3, 130])
def test_mlp_gradients_match_oracle(P, n):
    """FP32 gradients on the GPU against the FP64 oracle, per tensor in norm"""
    w = random_weights(12)
    rng = np.random.default_rng(13 + n)
    x = rng.uniform(-1, 1, (n, 7)).astype(np.float32)
    y = rng.normal(0.5, 1.0, (n, 256)).astype(np.float32)
    with P.Context() as c:
        loss, g = c.mlp_loss_grad(w, x, y)
    lref, gref = O.mlp_loss_grad(w.astype(np.float64), x.astype(np.float64), y.astype(np.float64))
    assert abs(loss - lref) <= 1e-5 * lref
    for name, sl in layer_slices():
        err = np.linalg.norm(g[sl] - gref[sl]) / np.linalg.norm(gref[sl])
        assert err <= 1e-4, (name, err)


def test_adam_matches_oracle(P, torch):
    rng = np.random.default_rng(14)
    np_ = O.mlp_nparams()
    w0 = rng.normal(0, 1, np_)
    with P.Context() as c:
        w = torch.tensor(w0, dtype=torch.float32, device="cuda")
        m = torch.zeros_like(w)
        v = torch.zeros_like(w)
        wr, mr, vr = w0.astype(np.float32).astype(np.float64), np.zeros(np_), np.zeros(np_)
        for t in range(1, 5):
            g0 = rng.normal(0, 1e-2, np_).astype(np.float32)
            g = torch.tensor(g0, device="cuda")
            c.mlp_adam(w, g, m, v, t, 1e-3)
            O.mlp_adam(wr, g0.astype(np.float64), mr, vr, t, 1e-3)
            torch.cuda.synchronize()
            assert np.abs(w.cpu().numpy() - wr).max() <= 2e-6
            assert np.abs(m.cpu().numpy() - mr).max() <= 1e-8


def test_training_graph_replays_match_eager_launches(P):
    """One captured step replayed per iteration gives bit-identical weights and
    the same minibatch losses as launching the kernels one by one."""
    rng = np.random.default_rng(15)
    x = rng.uniform(-1, 1, (700, 7)).astype(np.float32)
    y = (np.sin(x[:, :1] * np.arange(256) / 40.0) + x[:, 1:2]).astype(np.float32)
    with P.Context() as c:
        wg, hg = c.seed_train(x, y, steps=120, batch=96, use_graph=1, seed=5)
        we, he = c.seed_train(x, y, steps=120, batch=96, use_graph=0, seed=5)
    assert np.array_equal(wg, we)
    assert np.array_equal(hg, he)
    assert hg[-10:].mean() < 0.3 * hg[:10].mean()


# ------------------------------------------------------------------ features, labels
def small_case():
    cfg = W.config("C1")
    q = np.array([[0.3, 0.2], [-2.6, 0.9], [2.2, -2.9], [-0.7, -1.9], [3.4, 0.5], [-1.0, 7.1],
                  [math.pi, 0.0], [0.0, -math.pi]])
    return cfg, q


def test_features_match_oracle(P):
    cfg, q = small_case()
    params = np.array([[1.0, -0.2, -0.6, 0.07, 0.4], [2.0, 0.0, 0.3, 0.1, 3.0]])
    n = len(params) * len(q) * 2
    feat = np.zeros((n, 7), dtype=np.float32)
    lab = np.zeros((n, 256), dtype=np.float32)
    with P.Context(max_regions=1 << 14, max_active=64) as c:
        c.set_label_output(feat, lab)
        c.integrate(params, q, cfg["ff"], cfg["L"], rtol=1e-3)
    k = 0
    for p in params:
        for l in q:
            for och in (O.PP, O.PH):
                ref, _ = O.seed_features(p[0], p[1], p[2], p[3], p[4], l[0], l[1], och)
                assert np.abs(feat[k] - ref).max() <= 1e-6, (k, feat[k], ref)
                assert np.all(lab[k] > 0)
                k += 1


def test_labels_match_oracle_trees(P):
    """Labels of converged trees.  The device's selection takes leaves of the
    top key bin (a factor 2^(1/4) wide) in index order, not in exact key
    order, so its trees differ from the oracle's in places; labels of known
    trees are checked exactly by the seed-tree test below.  Checked here: the
    labels count exactly the leaves the device reports, and in the model
    frame they agree with the oracle's trees in almost every cell (a wrong
    frame map would move most of them)."""
    cfg, q = small_case()
    q = q[:4]
    p = cfg["params"][0]
    n = len(q) * 2
    lab = np.zeros((n, 256), dtype=np.float32)
    with P.Context(max_regions=1 << 14, max_active=16, batch=1, batch_max=1) as c:
        c.set_label_output(None, lab)
        _, _, st, _ = c.integrate(cfg["params"], q, cfg["ff"], cfg["L"], rtol=1e-4)
    k = 0
    ndiff = []
    for l in q:
        for och in (O.PP, O.PH):
            cont = O.Container(cfg["ff"], cfg["L"], t=p[0], tp=p[1], mu=p[2], T=p[3], Omega=p[4],
                               lx=l[0], ly=l[1], channel=och)
            _, _, ost, y = cont.integrate_labels(rtol=1e-4, batch=1)
            _, cm = O.seed_features(*p, l[0], l[1], och)
            ym = np.zeros(256)
            ym[cm] = y
            ndiff.append(int(np.sum(np.abs(lab[k] - ym) > 1e-6)))
            assert np.mean(np.abs(lab[k] - ym)) <= 0.1, k
            k += 1
    assert max(ndiff) <= 40 and sum(ndiff) <= 8 * 20, ndiff
    leaves = np.sum(np.exp2(lab.astype(np.float64)) - 1.0)
    assert abs(leaves - st["regions"]) <= 1e-5 * st["regions"], (leaves, st["regions"])


# ------------------------------------------------------------------ seed trees
def constant_model(ynet, seed=16):
    """a model whose output is ynet for every input: last layer W = 0, b = ynet"""
    w = random_weights(seed)
    sl = dict(layer_slices())
    w[sl["W4"]] = 0.0
    w[sl["b4"]] = ynet
    return w


@pytest.mark.parametrize("case", ["moderate", "deep", "limited"])
def test_seed_tree_and_sums_match_oracle(P, case):
    """With atol huge the adaptive loop stops as soon as the seed phase ends, so
    the final tree is the seed tree: its labels must be the oracle seed tree's,
    and the values the oracle's sums of Q_2N over its leaves (this checks that
    every placeholder was split and nothing was counted twice)."""
    rng = np.random.default_rng({"moderate": 20, "deep": 21, "limited": 22}[case])
    lo, hi = {"moderate": (0.0, 3.5), "deep": (1.0, 6.0), "limited": (1.0, 6.0)}[case]
    ynet = rng.uniform(lo, hi, 256).astype(np.float32)
    cap = 1 << 12 if case == "limited" else 1 << 16
    dmax = 8
    kappa = 1.5
    cfg, q = small_case()
    q = q[[0, 1, 4, 5]]
    p = np.array([[1.0, -0.2, -0.6, 0.07, 0.4]])
    n = len(q) * 2
    lab = np.zeros((n, 256), dtype=np.float32)
    with P.Context(max_regions=cap, max_active=8) as c:
        c.set_seed_model(constant_model(ynet), dmax=dmax, kappa=kappa)
        c.set_label_output(None, lab)
        out, _, st, rc = c.integrate(p, q, cfg["ff"], cfg["L"], rtol=1e-6, atol=1e300)
    assert st["seeded"] == n
    out = out.reshape(n, 5, 5)
    k = 0
    depths = []
    for l in q:
        for och in (O.PP, O.PH):
            x, cm = O.seed_features(*p[0], l[0], l[1], och)
            count = np.maximum(np.exp2(ynet[cm].astype(np.float64)) - 1.0, 0.0)
            nl, rects, D = O.seed_tree(count, dmax, 4 * kappa, cap // 4)
            depths.append(D)
            ym = np.zeros(256)
            ym[cm] = O.tree_labels(rects)
            assert np.abs(lab[k] - ym).max() <= 1e-6, (k, nl)
            cont = O.Container(cfg["ff"], cfg["L"], t=p[0][0], tp=p[0][1], mu=p[0][2], T=p[0][3],
                               Omega=p[0][4], lx=l[0], ly=l[1], channel=och)
            tot = np.zeros(15)
            for r in rects:
                tot += cont.region(*r)[1]
            ref = np.zeros((5, 5))
            ref[np.triu_indices(5)] = tot
            ref = ref + np.triu(ref, 1).T
            assert np.abs(out[k] - ref).max() <= 1e-11 * np.abs(ref).max(), k
            k += 1
    if case == "limited":
        assert max(depths) < dmax
    else:
        assert max(depths) >= 4


def test_seeded_integration_meets_the_gate(P):
    """Seeding from an untrained model changes the tree, not the answer: the
    adaptive loop still delivers the oracle's values within the gate."""
    cfg = dict(ff=W.ff_box(1), L=1)
    prm = np.array([(1, -0.2, -0.5, 0.05, 0.3), (1, -0.3, -1.0, 0.03, 0.05),
                    (1, -0.1, -0.2, 0.08, 2.0)], dtype=np.float64)
    q = W.q_grid(16)[::53][:4]
    with P.Context(max_regions=1 << 18, max_active=64) as c:
        c.set_seed_model(random_weights(17, scale=2.0), kappa=1.0)
        out, _, st, rc = c.integrate(prm, q, cfg["ff"], cfg["L"], rtol=1e-6)
    assert rc == 0 and st["seeded"] > 0
    picks = [(ip, iq, ch) for ip in range(len(prm)) for iq in range(len(q)) for ch in (O.PP, O.PH)]
    conts = [O.Container(cfg["ff"], cfg["L"], t=prm[ip][0], tp=prm[ip][1], mu=prm[ip][2],
                         T=prm[ip][3], Omega=prm[ip][4], lx=q[iq][0], ly=q[iq][1], channel=ch)
             for ip, iq, ch in picks]
    ref, _, _, nc = O.integrate_batch(conts, rtol=1e-9, err_mode=O.ERR_GLOBAL, batch=4,
                                      nthreads=THREADS)
    assert nc == 0
    gpu = out.reshape(len(picks), *out.shape[-2:])
    worst = max(gate_ratio(gpu[k], ref[k], 1e-6) for k in range(len(picks)))
    assert worst <= 1.0, worst


# ------------------------------------------------------------------ gain
def test_trained_model_saves_evaluations(P):
    """Train the model on trees the library itself produced (random parameter
    rows of the batched workload's distribution, q on the 16x16 grid), then
    integrate held-out rows both ways: the seeded run must need fewer
    integrand evaluations, and both must agree within the gate."""
    rng = np.random.default_rng(30)
    ff = W.ff_box(1)
    grid = W.q_grid(16)

    def rows(n):
        return np.stack([np.ones(n), rng.uniform(-0.35, 0.0, n), rng.uniform(-1.2, 0.0, n),
                         np.exp(rng.uniform(math.log(0.005), math.log(0.1), n)),
                         np.exp(rng.uniform(math.log(0.01), math.log(10.0), n))], axis=1)

    xs, ys = [], []
    with P.Context(max_regions=1 << 16) as c:
        for call in range(6):
            prm = rows(16)
            q = grid[rng.choice(len(grid), 24, replace=False)]
            n = len(prm) * len(q) * 2
            f = np.zeros((n, 7), dtype=np.float32)
            y = np.zeros((n, 256), dtype=np.float32)
            c.set_label_output(f, y)
            c.integrate(prm, q, ff, 1, rtol=1e-6)
            xs.append(f)
            ys.append(y)
        c.set_label_output(None, None)
        x = np.concatenate(xs)
        y = np.concatenate(ys)
        w, hist = c.seed_train(x, y, steps=1500, batch=256, seed=3)
        assert hist[-100:].mean() < 0.5 * hist[:20].mean()
        prm = rows(4)
        q = grid[rng.choice(len(grid), 32, replace=False)]
        plain, _, sp, _ = c.integrate(prm, q, ff, 1, rtol=1e-6)
        c.set_seed_model(w)
        seeded, _, ss, _ = c.integrate(prm, q, ff, 1, rtol=1e-6)
    print(f"\nevaluations plain {sp['kernel_evals']:.4g} seeded {ss['kernel_evals']:.4g} "
          f"({ss['kernel_evals'] / sp['kernel_evals']:.3f}); regions {sp['regions']} vs "
          f"{ss['regions']}; time {sp['seconds']:.3f} s vs {ss['seconds']:.3f} s")
    assert ss["kernel_evals"] < sp["kernel_evals"]
    a = plain.reshape(-1, 9, 9)
    b = seeded.reshape(-1, 9, 9)
    worst = max(gate_ratio(b[k], a[k], 2e-6) for k in range(len(a)))
    assert worst <= 1.0, worst
