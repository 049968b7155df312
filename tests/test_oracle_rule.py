"""Pins of the oracle's building blocks: the Clenshaw-Curtis pair (Sec. 3),
the Hurwitz zeta used for the frequency-sum tail, the dispersion (Sec. 2)
and the box basis of form factors (Sec. 2, truncated orthonormal basis)."""
import math
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_cc_weights_n4_match_textbook_fractions():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "cc_weights_n4.txt"))
            if l.strip() and not l.startswith("#")]
    x, w = O.cc_rule(4)
    for k, num, den in rows:
        assert abs(w[int(k)] - float(Fraction(int(num), int(den)))) < 1e-15
    assert np.allclose(x, np.cos(np.arange(5) * np.pi / 4), atol=1e-16)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 12, 16])
def test_cc_exact_degree_and_positivity(n):
    x, w = O.cc_rule(n)
    assert abs(w.sum() - 2.0) < 1e-14
    assert (w > 0).all()
    # exact through degree n (n+1 for even n, by symmetry)
    top = n + 1 if n % 2 == 0 else n
    for k in range(top + 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14, k
    # and not exact one degree higher for even degrees (a real check of order)
    k = top + 1 if (top + 1) % 2 == 0 else top + 2
    assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-11


@pytest.mark.parametrize("n", [2, 4, 6, 8])
def test_cc_nesting_is_bitwise(n):
    x1, _ = O.cc_rule(n)
    x2, _ = O.cc_rule(2 * n)
    assert np.array_equal(x1, x2[::2])
    assert x2[n] == 0.0 and np.array_equal(x2, -x2[::-1])


def test_hurwitz_zeta_against_direct_sums():
    mp.mp.dps = 40
    for s in [2, 4, 6, 10, 24, 48]:
        for q in [0.5, 3.5, 40.5, 800.5]:
            ref = mp.fsum((mp.mpf(q) + j) ** (-s) for j in range(20000))
            Q = mp.mpf(q) + 20000  # tail beyond the direct terms (Euler-Maclaurin, 3 terms)
            ref += Q ** (1 - s) / (s - 1) + Q ** (-s) / 2 + s * Q ** (-s - 1) / 12
            got = O.hurwitz_zeta(s, q)
            assert abs(got - float(ref)) <= 2e-15 * float(ref), (s, q)
    # classical value: zeta(2, 1/2) = pi^2/2
    assert abs(O.hurwitz_zeta(2, 0.5) - math.pi ** 2 / 2) < 1e-14


def test_dispersion_special_points():
    t, tp, mu = 1.0, -0.25, -0.95
    assert abs(O.dispersion(t, tp, mu, 0, 0) - (-4 * t - 4 * tp - mu)) < 1e-15
    assert abs(O.dispersion(t, tp, mu, math.pi, 0) - (4 * tp - mu)) < 1e-15
    assert abs(O.dispersion(t, tp, mu, math.pi, math.pi) - (4 * t - 4 * tp - mu)) < 1e-15
    # van Hove level at (pi, 0) is 4t' - mu
    assert abs(O.dispersion(1, 0, 0, 1.0, 2.0) - (-2 * (math.cos(1) + math.cos(2)))) < 1e-15


def test_box_basis_values_and_orthonormality():
    L = 2
    u = O.box_basis(L, 0.7)
    s2 = math.sqrt(2)
    assert np.allclose(u, [1, s2 * math.cos(0.7), s2 * math.sin(0.7), s2 * math.cos(1.4),
                           s2 * math.sin(1.4)], atol=1e-15)
    # discrete orthonormality on a uniform periodic grid (exact for these frequencies)
    xs = -math.pi + 2 * math.pi * (np.arange(64) + 0.5) / 64
    U = np.array([O.box_basis(L, x) for x in xs])
    G = U.T @ U / 64
    assert np.allclose(G, np.eye(2 * L + 1), atol=1e-14)
