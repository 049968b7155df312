"""Pins of the oracle's contraction (Sec. 2, Eqs. matmul-P/C/D) by algebra:
identity couplings, equal C and D couplings, single-entry couplings (closed
form of the cross terms, which a transposed or swapped product fails),
symmetry and homogeneity."""
import numpy as np

import oracle


def rnd(rng, n_l, M, sym=False):
    a = rng.normal(size=(n_l, M, M))
    return 0.5 * (a + a.transpose(0, 2, 1)) if sym else a


def test_identity_couplings_return_the_bubbles():
    rng = np.random.default_rng(1)
    chi = rng.normal(size=(3, 2, 5, 5))
    I = np.broadcast_to(np.eye(5), (3, 5, 5))
    dP, dC, dD = oracle.contract(chi, I, I, I)
    assert np.array_equal(dP, chi[:, 0])
    assert np.array_equal(dC, -chi[:, 1])
    assert np.abs(dD).max() == 0.0


def test_equal_c_and_d_couplings_cancel_in_d():
    rng = np.random.default_rng(2)
    chi = rng.normal(size=(4, 2, 9, 9))
    V = rnd(rng, 4, 9)
    _, dC, dD = oracle.contract(chi, rnd(rng, 4, 9), V, V)
    assert np.abs(dD).max() <= 1e-13 * np.abs(dC).max()


def test_single_entry_couplings_closed_form():
    """V^C = E_ij, V^D = E_kl: V^C chi V^D = chi_jk E_il, V^D chi V^C = chi_li E_kj,
    V^D chi V^D = chi_lk E_kl, V^C chi V^C = chi_ji E_ij."""
    rng = np.random.default_rng(3)
    M = 6
    chi = rng.normal(size=(1, 2, M, M))
    ph = chi[0, 1]
    i, j, k, l = 1, 4, 2, 5
    E = lambda a, b: np.eye(M)[:, [a]] @ np.eye(M)[[b], :]
    VC, VD = E(i, j)[None], E(k, l)[None]
    VP = E(j, i)[None]
    dP, dC, dD = oracle.contract(chi, VP, VC, VD)
    assert np.array_equal(dP[0], chi[0, 0][i, j] * E(j, i))
    assert np.array_equal(dC[0], -ph[j, i] * E(i, j))
    expect = 2 * ph[l, k] * E(k, l) - ph[j, k] * E(i, l) - ph[l, i] * E(k, j)
    assert np.array_equal(dD[0], expect)


def test_symmetry_and_homogeneity():
    rng = np.random.default_rng(4)
    chi = np.stack([rnd(rng, 2, 7, True), rnd(rng, 2, 7, True)], axis=1)
    VP, VC, VD = (rnd(rng, 2, 7, True) for _ in range(3))
    dP, dC, dD = oracle.contract(chi, VP, VC, VD)
    for X in (dP, dC, dD):
        assert np.abs(X - X.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(X).max()
    s = 1.7
    sP, sC, sD = oracle.contract(2.0 * chi, s * VP, s * VC, s * VD)
    for a, b in ((sP, dP), (sC, dC), (sD, dD)):
        assert np.allclose(a, 2.0 * s * s * b, rtol=1e-13, atol=1e-13 * np.abs(b).max())
