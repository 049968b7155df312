"""Pins of the oracle's frequency-summed kernel K(a, b).

K is T sum_n over Matsubara frequencies of the Omega-derivative of the
regulated product theta^2 G G (Sec. 2 and Eqs. chi_pp, chi_ph).  The oracle
sums a head of frequencies and expands the tail; these tests pin it to
things that do not share that construction:
  * a 30-digit mpmath sum of the same series (Euler-Maclaurin on the
    summand itself), on an adversarial grid of near-coincident energies;
  * the zero-temperature closed form, derived by contour integration;
  * the Lindhard function, which the Omega-integral of K must reproduce
    (theta -> 1 at Omega = 0 and -> 0 at Omega = infinity);
  * a central difference in Omega of the non-differentiated bubble;
  * the pp/ph relation G(-w, e) = -G(w, -e).
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import oracle as O


def k_mp(a, b, Om, T, ch, kind=O.BUBBLE_DOT):
    mp.mp.dps = 30
    a, b, Om, T = (mp.mpf(repr(v)) for v in (a, b, Om, T))

    def term(n):
        w = (2 * n + 1) * mp.pi * T
        u = w * w
        W = -4 * Om * u * u / (u + Om ** 2) ** 3 if kind == O.BUBBLE_DOT else u * u / (u + Om ** 2) ** 2
        P = (a * b - u) if ch == O.PH else (u + a * b)
        return W * P / ((u + a * a) * (u + b * b))

    big = max(abs(a), abs(b), Om, mp.pi * T)
    N = int(mp.ceil(20 * big / (2 * mp.pi * T))) + 10
    head = mp.fsum(term(n) for n in range(N))
    return float(2 * T * (head + mp.sumem(term, [N, mp.inf])))


def _adversarial_points():
    pts = []
    for T, Om in [(0.005, 0.01), (0.01, 0.1), (0.1, 1.0), (0.01, 10.0)]:
        for k in (1, 4, 8, 13):
            d = 10.0 ** -k
            pts += [(Om * (1 + d), Om * (1 - d), Om, T),      # both at +Omega
                    (Om * (1 + d), -Om, Om, T),               # +Omega and -Omega
                    (0.37 * (1 + d), 0.37, Om, T),            # a = b
                    (0.37 * (1 + d), -0.37, Om, T),           # a = -b
                    (d * T, -2 * d * T, Om, T)]               # both at the Fermi level
        pts += [(5.9, -6.1, Om, T), (0.0, 0.0, Om, T)]
    return pts


@pytest.mark.parametrize("pt", _adversarial_points())
def test_kernel_matches_high_precision_sum(pt):
    a, b, Om, T = pt
    for ch in (O.PP, O.PH):
        ref = k_mp(a, b, Om, T, ch)
        got = O.kernel(a, b, Om, T, ch)
        scale = max(abs(ref), abs(k_mp(abs(a) + 0.5 * T, abs(a) + 0.5 * T, Om, T, O.PH)))
        assert abs(got - ref) <= 1e-13 * scale, (ch, got, ref)


@pytest.mark.parametrize("pt", [(0.3, -0.7, 0.1, 0.1), (0.02, 0.05, 0.01, 0.005),
                                (2.0, 1.0, 1.0, 0.05)])
def test_bubble_kind_matches_high_precision_sum(pt):
    a, b, Om, T = pt
    for ch in (O.PP, O.PH):
        ref = k_mp(a, b, Om, T, ch, O.BUBBLE)
        assert abs(O.kernel(a, b, Om, T, ch, O.BUBBLE) - ref) <= 1e-13 * abs(ref)


def s0(x, Om):
    """Zero-temperature S(x) = int dw/2pi dtheta^2/dOmega / (i w - x): by
    contour integration x (3x + Omega) / (4 (x + Omega)^3) for x > 0, odd."""
    ax = abs(x)
    return math.copysign(ax * (3 * ax + Om) / (4 * (ax + Om) ** 3), x)


@pytest.mark.parametrize("a,b,Om", [(0.3, -0.7, 0.1), (0.5, 0.2, 1.0), (-1.5, -0.4, 0.25),
                                    (2.0, 2.0 + 1e-3, 0.7), (0.11, 0.09, 0.1)])
def test_zero_temperature_limit(a, b, Om):
    T = 5e-4  # exponentially close to T = 0 for energies >> T
    # ph: partial fractions 1/((iw-a)(iw-b)) = [1/(iw-a) - 1/(iw-b)]/(a-b)
    ph = (s0(a, Om) - s0(b, Om)) / (a - b)
    # pp: 1/((iw-a)(-iw-b)) = -[1/(iw-a) - 1/(iw+b)]/(a+b)
    pp = -(s0(a, Om) - s0(-b, Om)) / (a + b)
    assert abs(O.kernel(a, b, Om, T, O.PH) - ph) <= 1e-10 * abs(ph)
    assert abs(O.kernel(a, b, Om, T, O.PP) - pp) <= 1e-10 * abs(pp)


def lindhard(a, b, T, ch):
    if ch == O.PH:
        if a == b:
            f = O.fermi(a, T)
            return -f * (1 - f) / T
        return (O.fermi(a, T) - O.fermi(b, T)) / (a - b)
    return (1 - O.fermi(a, T) - O.fermi(b, T)) / (a + b)


@pytest.mark.parametrize("a,b,T", [(0.3, -0.7, 0.1), (0.05, 0.05, 0.05), (1.1, 0.4, 0.2)])
def test_omega_integral_is_bubble_minus_lindhard(a, b, T):
    """int_0^Oc dK/dOmega dOmega = K0(Oc) - K0(0), and K0(0) is the Lindhard
    function (theta = 1 at Omega = 0)."""
    Oc = 2.0
    for ch in (O.PP, O.PH):
        f = lambda s: O.kernel(a, b, math.exp(s), T, ch) * math.exp(s)
        val = sum(integrate.quad(f, lo, hi, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
                  for lo, hi in [(-40, -8), (-8, -3), (-3, math.log(Oc))])
        ref = O.kernel(a, b, Oc, T, ch, O.BUBBLE) - lindhard(a, b, T, ch)
        assert abs(val - ref) <= 1e-9 * abs(lindhard(a, b, T, ch)), (ch, val, ref)


def test_bubble_vanishes_at_large_scale():
    """Omega -> infinity: theta^2 removes all frequencies below Omega and
    Omega K0 -> -/+ (1/2pi) int dw w^2/(w^2+1)^2 = -/+ 1/4 (ph/pp), with
    corrections of relative order (a^2+b^2)/Omega^2."""
    for ch, lim in ((O.PH, -0.25), (O.PP, 0.25)):
        d = [abs(O.kernel(0.3, -0.5, Om, 0.1, ch, O.BUBBLE) * Om - lim) for Om in (100.0, 400.0)]
        assert d[1] < 2e-6 and 10 < d[0] / d[1] < 22


def test_bubble_at_zero_scale_is_lindhard():
    for a, b, T in [(0.3, -0.7, 0.1), (0.05, 0.2, 0.02)]:
        for ch in (O.PP, O.PH):
            got = O.kernel(a, b, 1e-10, T, ch, O.BUBBLE)
            assert abs(got - lindhard(a, b, T, ch)) < 1e-8 * abs(lindhard(a, b, T, ch))


@pytest.mark.parametrize("a,b,Om,T", [(0.3, -0.7, 0.1, 0.1), (0.02, 0.05, 0.03, 0.01),
                                      (1.0, 1.2, 2.0, 0.05)])
def test_dot_is_omega_derivative_of_bubble(a, b, Om, T):
    for ch in (O.PP, O.PH):
        h = 1e-4 * Om
        fd = (O.kernel(a, b, Om + h, T, ch, O.BUBBLE) - O.kernel(a, b, Om - h, T, ch, O.BUBBLE)) / (2 * h)
        assert abs(fd - O.kernel(a, b, Om, T, ch)) <= 1e-6 * abs(fd)


def test_vanishes_linearly_at_small_scale():
    for ch in (O.PP, O.PH):
        r1 = O.kernel(0.3, -0.2, 1e-6, 0.05, ch) / 1e-6
        r2 = O.kernel(0.3, -0.2, 1e-7, 0.05, ch) / 1e-7
        assert abs(r1 - r2) <= 1e-4 * abs(r1)


def test_channel_relation_and_symmetry():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, b = rng.uniform(-3, 3, 2)
        Om, T = math.exp(rng.uniform(-4, 1)), math.exp(rng.uniform(-5, -2))
        pp = O.kernel(a, b, Om, T, O.PP)
        ph_m = O.kernel(a, -b, Om, T, O.PH)
        assert abs(pp + ph_m) <= 1e-13 * max(abs(pp), 1e-300)
        for ch in (O.PP, O.PH):
            assert abs(O.kernel(a, b, Om, T, ch) - O.kernel(b, a, Om, T, ch)) <= 1e-14 * abs(
                O.kernel(a, b, Om, T, ch))
