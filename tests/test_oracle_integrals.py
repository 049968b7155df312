"""Pins of the oracle's adaptive integration (Alg. 1, Alg. 2, Listings 1-5)
and of the integrals it computes (Eqs. chi_pp, chi_ph with the Omega-dot).

Independent references: brute-force periodic grids (exponentially convergent
for these analytic periodic integrands), closed forms (unit integrand,
Gaussian, constant dispersion, the q=0 Fermi-derivative limit), and exact
invariants of the lattice (point group, gauge shift by a reciprocal vector,
perfect nesting)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
import workloads as W

FF5, FF9, FF25 = W.ff5(), W.ff_box(1), W.ff_box(2)


def cont(ff, L, **kw):
    return O.Container(ff, L, **kw)


@pytest.mark.parametrize("ff,L", [(FF5, 1), (FF9, 1), (FF25, 2)])
def test_unit_integrand_gives_identity(ff, L):
    c = cont(ff, L, kind=O.UNIT)
    v, e, st = c.integrate(rtol=1e-12, atol=1e-13, err_mode=O.ERR_GLOBAL)
    assert st["converged"] == 1
    assert np.abs(v - np.eye(len(ff))).max() < 1e-12


def test_region_rule_pair_on_polynomials():
    """On a rectangle both rules of the pair integrate the constant exactly:
    area / (2 pi)^2 with the zone measure."""
    c = cont(FF9[:1], 1, kind=O.UNIT)
    qn, q2n = c.region(-0.3, 0.9, 0.1, 0.6)
    area = 1.2 * 0.5 / (4 * math.pi ** 2)
    assert abs(q2n[0] - area) < 1e-16 and abs(qn[0] - area) < 1e-16


def gauss_exact(x0, y0, s):
    f = lambda c: special.ndtr((math.pi - c) / s) - special.ndtr((-math.pi - c) / s)
    return 2 * math.pi * s * s * f(x0) * f(y0) / (4 * math.pi ** 2)


@pytest.mark.parametrize("x0,y0,s", [(0.3, -1.1, 0.4), (2.9, 0.0, 0.05), (-3.0, 3.1, 0.2)])
def test_gaussian_closed_form_and_honest_error(x0, y0, s):
    c = cont(FF9[:1], 1, kind=O.GAUSS, gauss=(x0, y0, s))
    for rtol in (1e-4, 1e-8, 1e-11):
        v, e, st = c.integrate(rtol=rtol, err_mode=O.ERR_GLOBAL)
        ex = gauss_exact(x0, y0, s)
        assert st["converged"] == 1
        assert abs(v[0, 0] - ex) <= max(e[0, 0], 1e-15)      # the estimate bounds the error
        assert abs(v[0, 0] - ex) <= rtol * abs(ex)


BASE = dict(t=1.0, tp=-0.25, mu=-0.95, T=0.2, Omega=0.3)


@pytest.mark.parametrize("ch", [O.PP, O.PH])
def test_adaptive_matches_brute_force_grid(ch):
    c = cont(FF9, 1, lx=1.57, ly=1.31, channel=ch, **BASE)
    b1, b2 = c.brute(192), c.brute(256)
    assert np.abs(b1 - b2).max() < 1e-13          # the grid itself has converged
    v, e, st = c.integrate(rtol=1e-10, err_mode=O.ERR_GLOBAL)
    assert st["converged"] == 1
    assert np.abs(v - b2).max() < 1e-11 * np.abs(b2).max()
    # both modes of task granularity agree (one task = region vs (region, pair))
    va, _, sta = cont(FF9, 1, lx=1.57, ly=1.31, channel=ch, **BASE).integrate(
        rtol=1e-9, mode=O.MODE_A, err_mode=O.ERR_GLOBAL)
    assert sta["converged"] == 1
    assert np.abs(va - b2).max() < 1e-9 * np.abs(b2).max()


def test_constant_dispersion_gives_diagonal():
    """t = t' = 0: eps = -mu everywhere, g is the constant K(-mu, -mu)."""
    mu = 0.13
    for ch in (O.PP, O.PH):
        c = cont(FF9, 1, t=0.0, tp=0.0, mu=mu, T=0.05, Omega=0.07, lx=0.4, ly=2.0, channel=ch)
        v, e, st = c.integrate(rtol=1e-11, err_mode=O.ERR_GLOBAL)
        k = O.kernel(-mu, -mu, 0.07, 0.05, ch)
        assert np.abs(v - k * np.eye(9)).max() < 1e-11 * abs(k)


def _xfreq_sign(L, axis):
    """(-1)^(frequency along the axis) for each box basis function."""
    nb = 2 * L + 1
    k = np.array([0] + [j for j in range(1, L + 1) for _ in (0, 1)])
    s = np.array([(-1.0) ** (k[a] if axis == 0 else k[b]) for a in range(nb) for b in range(nb)])
    return s


def _odd_sign(L, axis):
    """-1 for basis functions odd under p_axis -> -p_axis (a sine factor)."""
    nb = 2 * L + 1
    odd = [0] + [0 if j % 2 == 1 else 1 for j in range(1, 2 * L + 1)]
    return np.array([(-1.0) ** (odd[a] if axis == 0 else odd[b]) for a in range(nb) for b in range(nb)])


def _swap_perm(L):
    nb = 2 * L + 1
    return np.array([b * nb + a for a in range(nb) for b in range(nb)])


@pytest.mark.parametrize("ch", [O.PP, O.PH])
def test_lattice_invariants(ch):
    kw = dict(channel=ch, **BASE)
    opt = dict(rtol=1e-10, err_mode=O.ERR_GLOBAL)
    l = (1.1, 0.45)
    v, _, _ = cont(FF9, 1, lx=l[0], ly=l[1], **kw).integrate(**opt)
    tol = 1e-10 * np.abs(v).max()
    assert np.abs(v - v.T).max() == 0.0
    # inversion p -> -p leaves g invariant: pairs with an odd number of sines vanish
    par = _odd_sign(1, 0) * _odd_sign(1, 1)
    assert np.abs(v[np.outer(par, par) < 0]).max() < tol
    # mirror k_x -> -k_x
    vm, _, _ = cont(FF9, 1, lx=-l[0], ly=l[1], **kw).integrate(**opt)
    s = _odd_sign(1, 0)
    assert np.abs(vm - np.outer(s, s) * v).max() < tol
    # swap x <-> y
    vs, _, _ = cont(FF9, 1, lx=l[1], ly=l[0], **kw).integrate(**opt)
    P = _swap_perm(1)
    assert np.abs(vs - v[np.ix_(P, P)]).max() < tol
    # gauge: l -> l + 2 pi e_x shifts p by pi along x
    vg, _, _ = cont(FF9, 1, lx=l[0] + 2 * math.pi, ly=l[1], **kw).integrate(**opt)
    g = _xfreq_sign(1, 0)
    assert np.abs(vg - np.outer(g, g) * v).max() < tol


def test_perfect_nesting_relation():
    """t' = 0, mu = 0: eps(k + Q) = -eps(k) for Q = (pi, pi), so the ph integrand
    at l = Q equals minus the pp integrand at l = 0 after p -> p + Q/2."""
    kw = dict(t=1.0, tp=0.0, mu=0.0, T=0.1, Omega=0.2)
    opt = dict(rtol=1e-10, err_mode=O.ERR_GLOBAL)
    ph, _, _ = cont(FF9[:1], 1, lx=math.pi, ly=math.pi, channel=O.PH, **kw).integrate(**opt)
    pp, _, _ = cont(FF9[:1], 1, lx=0.0, ly=0.0, channel=O.PP, **kw).integrate(**opt)
    assert abs(ph[0, 0] + pp[0, 0]) < 1e-10 * abs(pp[0, 0])


@pytest.mark.slow
def test_q0_omega_integral_is_fermi_derivative():
    """int_0^inf chi_dot^ph_mn(q=0; Omega) dOmega = chi(Omega=inf) - chi(Omega=0)
    = - int d^2p/(2pi)^2 n_F'(eps) f_m f_n  (theta = 1 at Omega = 0, 0 at infinity)."""
    t, tp, mu, T = 1.0, -0.25, -0.95, 0.25
    Lg = 160
    xs = -math.pi + 2 * math.pi * (np.arange(Lg) + 0.5) / Lg
    kx, ky = np.meshgrid(xs, xs, indexing="ij")
    eps = -2 * t * (np.cos(kx) + np.cos(ky)) - 4 * tp * np.cos(kx) * np.cos(ky) - mu
    nF = 1 / (np.exp(eps / T) + 1)
    dnF = -nF * (1 - nF) / T
    f1 = np.sqrt(2) * np.cos(kx)                # u_1(p_x) u_0(p_y), box index 3
    ref00 = -dnF.mean()
    ref33 = -(dnF * f1 * f1).mean()
    ff = FF9[[0, 3]]

    def chidot(s):
        Om = math.exp(s)
        c = cont(ff, 1, t=t, tp=tp, mu=mu, T=T, Omega=Om, channel=O.PH)
        return c.brute(96) * Om

    xg, wg = np.polynomial.legendre.leggauss(48)
    tot = np.zeros((2, 2))
    for lo, hi in [(-25, -6), (-6, -1), (-1, 2), (2, 6), (6, 9)]:
        for x, w in zip(xg, wg):
            tot += 0.5 * (hi - lo) * w * chidot(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
    # Omega > e^9: chi_dot = C/Omega^2 (1 + O(Omega^-2)); the tail is Omega chi_dot(Omega)
    tot += chidot(9.0)
    assert abs(tot[0, 0] - ref00) < 1e-9 * abs(ref00)
    assert abs(tot[1, 1] - ref33) < 1e-9 * abs(ref33)


def test_batch_extraction_and_budget():
    c = cont(FF5, 1, lx=2.0, ly=0.5, channel=O.PH, **BASE)
    v1, e1, s1 = c.integrate(rtol=1e-8, err_mode=O.ERR_GLOBAL, batch=1)
    v7, e7, s7 = c.integrate(rtol=1e-8, err_mode=O.ERR_GLOBAL, batch=7)
    assert s1["converged"] == s7["converged"] == 1
    assert s7["regions"] >= s1["regions"]           # bulk extraction can only overshoot
    assert np.abs(v1 - v7).max() < 1e-8 * np.abs(v1).max()
    vb, eb, sb = c.integrate(rtol=1e-12, err_mode=O.ERR_GLOBAL, max_regions=40)
    assert sb["converged"] == 0 and sb["regions"] <= 40


def test_per_integral_mode_meets_each_tolerance():
    c = cont(FF9, 1, lx=1.57, ly=1.31, channel=O.PP, **BASE)
    ref = c.brute(256)
    rtol, nu = 1e-7, 1e-3
    v, e, st = c.integrate(rtol=rtol, nu=nu, err_mode=O.ERR_PER_INTEGRAL)
    tau = rtol * np.maximum(np.abs(v), nu * np.abs(v).max())
    assert (e <= tau * (1 + 1e-12)).all()
    assert (np.abs(v - ref) <= tau).all()


# ------------------------------------------------------------------ weighted global criterion
def _wcont(pair_w, **kw):
    ff = W.ff5()
    return O.Container(ff, 1, t=1.0, tp=-0.2, mu=-0.4, T=0.1, Omega=0.3, lx=1.1, ly=0.4,
                       channel=O.PH, pair_w=pair_w, **kw)


def test_weighted_criterion_with_unit_pair_weights_is_the_global_one():
    """pair weights 1 (w_pp = 1, w_pq = w_qp = 1/2) reproduce the global mode bit for bit"""
    Wm = np.full((5, 5), 0.5) + 0.5 * np.eye(5)
    v1, e1, s1 = _wcont(Wm).integrate(rtol=1e-6, err_mode=O.ERR_WEIGHTED, batch=4)
    v0, e0, s0 = _wcont(None).integrate(rtol=1e-6, err_mode=O.ERR_GLOBAL, batch=4)
    assert np.array_equal(v1, v0) and np.array_equal(e1, e0)
    assert s1["regions"] == s0["regions"]


def test_weighted_criterion_is_scale_invariant():
    rng = np.random.default_rng(8)
    Wm = O.weights_from_couplings(rng.normal(size=(5, 5)))
    a = _wcont(Wm).integrate(rtol=1e-6, err_mode=O.ERR_WEIGHTED, batch=4)
    b = _wcont(4.0 * Wm).integrate(rtol=1e-6, err_mode=O.ERR_WEIGHTED, batch=4)
    assert np.array_equal(a[0], b[0]) and a[2]["regions"] == b[2]["regions"]


def test_weighted_criterion_holds_against_a_tight_reference():
    """the weighted error of the result stays within rtol of the weighted sum;
    a weight on one entry alone refines for that integral only"""
    rng = np.random.default_rng(9)
    ref, _, _ = _wcont(None).integrate(rtol=1e-11, err_mode=O.ERR_GLOBAL, batch=8)
    iu = np.triu_indices(5)
    for Wm in (O.weights_from_couplings(rng.normal(size=(5, 5))), np.eye(5)[:, :1] @ np.eye(5)[:1, :]):
        pw = np.where(np.eye(5) > 0, Wm, Wm + Wm.T)[iu]
        v, _, st = _wcont(Wm).integrate(rtol=1e-6, err_mode=O.ERR_WEIGHTED, batch=4)
        err = np.sum(pw * np.abs(v[iu] - ref[iu]))
        assert err <= 1e-6 * np.sum(pw * np.abs(ref[iu]))
    _, _, sg = _wcont(None).integrate(rtol=1e-6, err_mode=O.ERR_GLOBAL, batch=4)
    assert st["regions"] < sg["regions"]


def test_oracle_leaves_tile_the_zone_and_sum_to_the_value(oracle_lib):
    """the leaves the oracle returns (mode B, MaxTask 1) cover the zone once
    (their areas add up to (2 pi)^2 and none overlaps another), their number
    is the leaf count of the statistics, each leaf's Q_2N is the rule applied
    to its rectangle, and their sum in creation order is the returned value"""
    O = oracle_lib
    ff = np.eye(9)
    c = O.Container(ff, 1, t=1.0, tp=-0.25, mu=-0.95, T=0.1, Omega=0.3, lx=1.07, ly=-2.31,
                    channel=O.PP)
    v, e, st, rects, q2n = c.integrate_leaves(rtol=1e-3)
    assert len(rects) == st["regions"] > 4
    w = rects[:, 1] - rects[:, 0]
    assert np.allclose(w, rects[:, 3] - rects[:, 2])
    assert abs(np.sum(w * w) - (2 * np.pi) ** 2) <= 1e-12
    # no overlap: leaves are quadtree cells, so two overlap only if one contains the other
    lo = np.round((rects[:, [0, 2]] + np.pi) / w[:, None]).astype(np.int64)
    d = np.round(np.log2(2 * np.pi / w)).astype(int)
    cells = set()
    for (ix, iy), dd in zip(lo, d):
        for a in range(dd + 1):
            anc = (a, ix >> (dd - a), iy >> (dd - a))
            assert anc not in cells or a == dd, "a leaf lies inside another leaf"
        cells.add((dd, ix, iy))
    assert len(cells) == len(rects)
    for k in (0, len(rects) // 2, len(rects) - 1):
        _, q = c.region(*rects[k])
        assert np.array_equal(q, q2n[k])
    iu = np.triu_indices(9)
    s = np.zeros(45)
    for row in q2n:
        s += row
    assert np.array_equal(s, v[iu])
