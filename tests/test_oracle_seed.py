"""Pins of the oracle's subdivision-density model (multilayer perceptron,
Adam), the tree labels, the model-frame features and the seed tree.

None of these objects is in the paper: they serve the learned seeding of the
initial partition that sits in front of the adaptive loop of Alg. 2.  Each
check compares against something other than the oracle itself: a library
routine (scipy's normal CDF for GELU), a linear-algebra identity, central
finite differences, Adam's closed form under a constant gradient, the count
of leaves, and the lattice symmetry of the integrand.
"""
import math

import numpy as np
import pytest
from scipy.stats import norm

import oracle
import workloads

IN, HID, OUT = oracle.MLP_IN, oracle.MLP_HID, oracle.MLP_OUT
DIMS = [IN, HID, HID, HID, OUT]


def split_params(w):
    """views W_l [out][in], b_l [out] of the flat parameter array"""
    out, off = [], 0
    for l in range(4):
        ni, no = DIMS[l], DIMS[l + 1]
        W = w[off:off + no * ni].reshape(no, ni)
        off += no * ni
        b = w[off:off + no]
        off += no
        out.append((W, b))
    assert off == w.size
    return out


def random_params(rng, scale=1.0):
    w = np.zeros(oracle.mlp_nparams())
    for W, b in split_params(w):
        W[...] = rng.normal(0.0, scale / math.sqrt(W.shape[1]), W.shape)
        b[...] = rng.normal(0.0, 0.1, b.shape)
    return w


def test_param_count():
    assert oracle.mlp_nparams() == sum(DIMS[l + 1] * (DIMS[l] + 1) for l in range(4)) == 67072


def test_forward_linear_regime():
    """With hidden pre-activations near +20, GELU(z) = z to double precision
    (z Phi(-z) ~ 1e-87), so the network is the affine chain W4(W3(W2(W1 x +
    b1) + b2) + b3) + b4.  Non-square W1 and W4 make a transposed layer or a
    misplaced bias fail."""
    rng = np.random.default_rng(1)
    w = np.zeros(oracle.mlp_nparams())
    layers = split_params(w)
    for l, (W, b) in enumerate(layers):
        W[...] = rng.uniform(-1, 1, W.shape) * (0.05 / W.shape[1])
        b[...] = 20.0 if l < 3 else rng.normal(0, 1, b.shape)
    x = rng.uniform(-1, 1, (5, IN))
    h = x.T
    for l, (W, b) in enumerate(layers):
        h = W @ h + b[:, None]
    y = oracle.mlp_forward(w, x)
    assert np.allclose(y, h.T, rtol=1e-13, atol=1e-12)


def test_forward_gelu_values():
    """A single path x0 -> h -> h -> h -> y with unit weights gives
    y = G(G(G(x0))) with G(z) = z Phi(z); Phi from scipy."""
    w = np.zeros(oracle.mlp_nparams())
    layers = split_params(w)
    layers[0][0][0, 0] = 1.0
    layers[1][0][0, 0] = 1.0
    layers[2][0][0, 0] = 1.0
    layers[3][0][:, 0] = 1.0
    G = lambda z: z * norm.cdf(z)
    for x0 in (-3.0, -0.7, 0.0, 0.4, 1.3, 5.0):
        x = np.zeros((1, IN))
        x[0, 0] = x0
        y = oracle.mlp_forward(w, x)
        assert np.allclose(y, G(G(G(x0))), rtol=1e-14, atol=1e-15)


def test_gradient_finite_differences():
    """Fourth-order central differences of the loss agree with the analytic
    gradient to 1e-7 (norm-wise) on every tensor."""
    rng = np.random.default_rng(2)
    w = random_params(rng)
    x = rng.uniform(-1, 1, (3, IN))
    y = rng.normal(0, 1, (3, OUT))
    loss, g = oracle.mlp_loss_grad(w, x, y)
    # the loss itself: mean of squared residuals
    r = oracle.mlp_forward(w, x) - y
    assert abs(loss - np.mean(r * r)) <= 1e-14 * loss
    h = 1e-4
    f = lambda wv: oracle.mlp_loss_grad(wv, x, y)[0]
    off = 0
    for l in range(4):
        ni, no = DIMS[l], DIMS[l + 1]
        for name, size in (("W", no * ni), ("b", no)):
            idx = off + rng.choice(size, size=min(size, 48), replace=False)
            fd = np.zeros(idx.size)
            for k, i in enumerate(idx):
                vals = []
                for s in (2, 1, -1, -2):
                    wp = w.copy()
                    wp[i] += s * h
                    vals.append(f(wp))
                fd[k] = (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)
            err = np.linalg.norm(fd - g[idx]) / np.linalg.norm(g[idx])
            assert err <= 1e-7, (l, name, err)
            off += size


def test_adam_constant_gradient_closed_form():
    """Under a constant gradient g, Adam's bias-corrected moments are g and
    g^2 at every step, so each step moves w by -lr g / (|g| + 1e-8)."""
    rng = np.random.default_rng(3)
    n = 257
    w0 = rng.normal(0, 1, n)
    g = rng.normal(0, 1e-3, n)
    g[0] = 0.0
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    lr = 0.01
    for t in range(1, 6):
        oracle.mlp_adam(w, g, m, v, t, lr)
        expect = w0 - t * lr * g / (np.abs(g) + 1e-8)
        assert np.allclose(w, expect, rtol=0, atol=1e-13)
    assert w[0] == w0[0]


def test_training_lowers_the_loss():
    rng = np.random.default_rng(4)
    w = random_params(rng)
    x = rng.uniform(-1, 1, (24, IN))
    y = np.tile(np.sin(np.arange(OUT) / 20.0), (24, 1)) * x[:, :1] + 0.5
    m, v = np.zeros_like(w), np.zeros_like(w)
    l0 = oracle.mlp_loss_grad(w, x, y)[0]
    for t in range(1, 61):
        loss, g = oracle.mlp_loss_grad(w, x, y)
        oracle.mlp_adam(w, g, m, v, t, 3e-3)
    l1 = oracle.mlp_loss_grad(w, x, y)[0]
    assert l1 < 0.1 * l0


# ------------------------------------------------------------------ labels
PI = math.pi


def quad_rect(d, i, j):
    w = 2 * PI / 2 ** d
    return [-PI + i * w, -PI + (i + 1) * w, -PI + j * w, -PI + (j + 1) * w]


def test_labels_root_and_uniform_trees():
    y = oracle.tree_labels([quad_rect(0, 0, 0)])
    assert np.allclose(y, math.log2(1 + 1 / 256), rtol=1e-15)
    y = oracle.tree_labels([quad_rect(4, i, j) for i in range(16) for j in range(16)])
    assert np.allclose(y, 1.0, rtol=1e-15)
    # four depth-5 leaves inside cell (3, 7), the rest of the zone empty
    y = oracle.tree_labels([quad_rect(5, 6 + a, 14 + b) for a in (0, 1) for b in (0, 1)])
    assert abs(y[16 * 7 + 3] - math.log2(5)) < 1e-14
    assert np.count_nonzero(y) == 1


def random_quadtree(rng, depth_max=7, p_split=0.6):
    leaves, stack = [], [(0, 0, 0)]
    while stack:
        d, i, j = stack.pop()
        if d < depth_max and rng.random() < (p_split if d else 1.0):
            stack += [(d + 1, 2 * i + a, 2 * j + b) for a in (0, 1) for b in (0, 1)]
        else:
            leaves.append(quad_rect(d, i, j))
    return leaves


def test_labels_count_leaves():
    """sum over cells of (2^y - 1) is the number of leaves"""
    rng = np.random.default_rng(5)
    for _ in range(5):
        leaves = random_quadtree(rng)
        y = oracle.tree_labels(leaves)
        assert abs(np.sum(2.0 ** y - 1.0) - len(leaves)) < 1e-9 * len(leaves)


# ------------------------------------------------------------------ features
def d4_images(lx, ly):
    out = []
    for sw in (0, 1):
        for sx in (1, -1):
            for sy in (1, -1):
                a, b = (ly, lx) if sw else (lx, ly)
                out.append((sx * a, sy * b))
    return out


def test_features_fold_and_cellmap_permutation():
    rng = np.random.default_rng(6)
    for _ in range(20):
        lx, ly = rng.uniform(-7, 7, 2)
        x, cm = oracle.seed_features(1.0, -0.2, -0.5, 0.02, 0.3, lx, ly, oracle.PP)
        assert 0 <= x[1] <= x[0] <= 1
        assert sorted(cm) == list(range(256))
        assert x[6] == -1.0 and abs(x[3] - math.log10(0.02)) < 1e-15
        for gx, gy in d4_images(lx, ly) + [(lx + 2 * PI, ly), (lx, ly - 4 * PI)]:
            x2, cm2 = oracle.seed_features(1.0, -0.2, -0.5, 0.02, 0.3, gx, gy, oracle.PP)
            assert np.allclose(x2, x, atol=1e-14)


def test_features_scale_with_hopping():
    x1, _ = oracle.seed_features(1.0, -0.2, -0.5, 0.02, 0.3, 0.4, 0.1, oracle.PH)
    x2, _ = oracle.seed_features(2.0, -0.4, -1.0, 0.04, 0.6, 0.4, 0.1, oracle.PH)
    assert np.allclose(x1, x2, atol=1e-14)


@pytest.mark.parametrize("l", [(1.1, 0.4), (-2.6, 0.9)])
def test_model_frame_labels_are_symmetric(l):
    """The integrand at g l is the integrand at l moved by g, and at
    l + 2 pi e_x it is moved by pi e_x; so the model-frame labels of the
    converged trees of all these momenta coincide (up to ties of equal keys,
    hence the small tolerance).  A wrong direction in the cell map fails."""
    ff = workloads.ff5()
    ref = None
    for gx, gy in d4_images(*l)[::3] + [(l[0] + 2 * PI, l[1])]:
        c = oracle.Container(ff, 1, t=1.0, tp=0.0, mu=-0.4, T=0.1, Omega=0.3, lx=gx, ly=gy,
                             channel=oracle.PH)
        _, _, st, y = c.integrate_labels(rtol=1e-3)
        _, cm = oracle.seed_features(1.0, 0.0, -0.4, 0.1, 0.3, gx, gy, oracle.PH)
        ym = np.zeros(256)
        ym[cm] = y
        if ref is None:
            ref = ym
            assert st["regions"] > 40
        else:
            assert np.mean(np.abs(ym - ref)) < 0.02, (gx, gy)


# ------------------------------------------------------------------ seed tree
def pyramid_leaves(count, D, thresh):
    """the seed rule on a sum pyramid of the cell counts (a second
    formulation: level d from level d+1 by 2x2 sums; depths > 4 scale by 1/4)"""
    lv = {4: count.reshape(16, 16)}
    for d in (3, 2, 1, 0):
        a = lv[d + 1]
        lv[d] = a[0::2, 0::2] + a[1::2, 0::2] + a[0::2, 1::2] + a[1::2, 1::2]
    n, stack = 0, [(0, 0, 0)]
    while stack:
        d, i, j = stack.pop()
        c = lv[d][j, i] if d <= 4 else lv[4][j >> (d - 4), i >> (d - 4)] / 4.0 ** (d - 4)
        if d < D and c >= thresh:
            stack += [(d + 1, 2 * i + a, 2 * j + b) for a in (0, 1) for b in (0, 1)]
        else:
            n += 1
    return n


def test_seed_tree_uniform_closed_form():
    # c per cell: depth-4 nodes hold c, deeper ones c/4^k; split while >= 8
    for c, expect in ((3.0, 256), (9.0, 1024), (40.0, 4096), (100.0, 4096), (200.0, 16384),
                      (0.01, 1), (0.04, 4)):
        n, rects, D = oracle.seed_tree(np.full(256, c), 9, 8.0, 10 ** 7)
        assert n == expect, (c, n)
        assert abs(sum((r[1] - r[0]) * (r[3] - r[2]) for r in rects) - 4 * PI * PI) < 1e-9


def test_seed_tree_matches_pyramid_rule_and_limit():
    rng = np.random.default_rng(7)
    for k in range(6):
        y = rng.normal(1.0, 1.5, 256)
        count = np.maximum(np.exp2(y) - 1.0, 0.0)
        n, rects, D = oracle.seed_tree(count, 8, 8.0, 10 ** 7)
        assert D == 8 and n == pyramid_leaves(count, 8, 8.0) == len(rects)
        lim = max(1, n // 3)
        n2, _, D2 = oracle.seed_tree(count, 8, 8.0, lim)
        assert n2 <= lim and D2 < 8
        assert pyramid_leaves(count, D2, 8.0) == n2
        assert D2 == 0 or pyramid_leaves(count, D2 + 1, 8.0) > lim
