"""GPU contraction (Eqs. matmul-P/C/D on the FP64 matrix cores) against the
oracle's definition, through the C ABI."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paid_1610_09991_amd as P
    c = P.Context()
    yield c
    c.close()


@pytest.mark.parametrize("M", [1, 5, 9, 16, 17, 25, 32])
@pytest.mark.parametrize("n_l", [1, 3, 70])
def test_contraction_matches_oracle(ctx, M, n_l):
    rng = np.random.default_rng(100 * M + n_l)
    chi = rng.normal(size=(n_l, 2, M, M))
    VP, VC, VD = (rng.normal(size=(n_l, M, M)) for _ in range(3))
    got = ctx.contract(chi, VP, VC, VD)
    ref = O.contract(chi, VP, VC, VD)
    for g, r in zip(got, ref):
        scale = np.abs(r).max(axis=(1, 2), keepdims=True)
        assert np.all(np.abs(g - r) <= 1e-13 * scale * M)


def test_contraction_of_device_tensors(ctx):
    import torch
    rng = np.random.default_rng(5)
    chi = rng.normal(size=(11, 2, 9, 9))
    V = [rng.normal(size=(11, 9, 9)) for _ in range(3)]
    tchi = torch.tensor(chi, device="cuda")
    tV = [torch.tensor(v, device="cuda") for v in V]
    got = ctx.contract(tchi, *tV)
    ref = O.contract(chi, *V)
    for g, r in zip(got, ref):
        assert np.abs(g.cpu().numpy() - r).max() <= 1e-12 * np.abs(r).max()


def test_integrate_then_contract_against_the_oracle_chain(ctx):
    """paid_integrate's output layout feeds paid_contract directly; the chain
    agrees with the oracle's own integration and contraction."""
    import paid_1610_09991_amd as P
    cfg = W.config("C1")
    q = cfg["q"][[3, 17, 40]]
    out, _, _, _ = ctx.integrate(cfg["params"], q, cfg["ff"], cfg["L"], P.PP | P.PH, rtol=1e-8)
    chi = out.reshape(len(q), 2, 5, 5)
    rng = np.random.default_rng(6)
    V = [rng.normal(size=(len(q), 5, 5)) for _ in range(3)]
    got = ctx.contract(chi, *V)
    p = cfg["params"][0]
    conts = [O.Container(cfg["ff"], cfg["L"], t=p[0], tp=p[1], mu=p[2], T=p[3], Omega=p[4],
                         lx=l[0], ly=l[1], channel=ch) for l in q for ch in (O.PP, O.PH)]
    vals, _, _, nc = O.integrate_batch(conts, rtol=1e-11, err_mode=O.ERR_GLOBAL, batch=4,
                                       nthreads=8)
    assert nc == 0
    ref = O.contract(vals.reshape(len(q), 2, 5, 5), *V)
    for g, r, v in zip(got, ref, (V[0], V[1], V[2])):
        # |error| <= |V| |d chi| |V| with |d chi| <= 1e-8 of the largest bubble
        bound = 1e-7 * np.abs(vals).max() * (np.abs(v).sum(axis=2).max() * np.abs(v).sum(axis=1).max() * 3)
        assert np.abs(g - r).max() <= bound


def test_contraction_rejects_bad_orders(ctx):
    import paid_1610_09991_amd as P
    z = np.zeros((1, 2, 33, 33))
    v = np.zeros((1, 33, 33))
    with pytest.raises(P.PaidError):
        ctx.contract(z, v, v, v)
