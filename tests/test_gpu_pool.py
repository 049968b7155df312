"""Two kinds of slots in the region pool (paid_config.small_regions): new
containers start in small slots and move, leaves and sums copied, to a large
slot of max_regions leaves when their next round could overflow the small
one.  A container never splits fewer leaves because of its small slot, so
the results must be bit-identical to those of one kind of slot of
max_regions (through the C ABI)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paid_1610_09991_amd as P
    P.lib()
    return P


def run(P, cfg, rows, nq, **kw):
    params = cfg["params"][rows]
    q = cfg["q"][:nq]
    with P.Context(graph=1, **kw) as ctx:
        out, err, st, rc = ctx.integrate(params, q, cfg["ff"], cfg["L"], rtol=cfg["rtol"],
                                         err=kw.get("err_mode", 0) == P.ERR_PER_INTEGRAL)
    assert rc == P.OK and st["not_converged"] == 0
    return out, err, st


@pytest.mark.parametrize("mode", ["global", "per_integral"])
@pytest.mark.parametrize("small,share", [(1 << 10, 0.25), (1 << 12, 0.0)])
def test_two_kinds_of_slots_match_one(P, mode, small, share):
    """C3 rows 0-5 (random T 0.005-0.1, Omega 0.01-1) at 16 q: most
    containers outgrow a small slot of 2^10 or 2^12 leaves and move; with
    big_share near 0 a single large slot serves them one after another"""
    cfg = W.config("C3")
    rows, nq = slice(0, 6), 16
    em = P.ERR_GLOBAL if mode == "global" else P.ERR_PER_INTEGRAL
    ref, eref, st1 = run(P, cfg, rows, nq, max_regions=1 << 19, err_mode=em)
    kw = dict(max_regions=1 << 19, err_mode=em, small_regions=small)
    if share:
        kw["big_share"] = share
    else:
        kw["big_share"] = 1e-9  # one large slot
    out, eout, st2 = run(P, cfg, rows, nq, **kw)
    print(f"{mode} small {small} share {share}: {st1['max_active']} -> {st2['max_active']} resident, "
          f"{st2['regions']} leaves, {st1['seconds']:.2f} -> {st2['seconds']:.2f} s")
    assert st2["regions"] == st1["regions"] and st2["splits"] == st1["splits"]
    assert np.array_equal(out, ref)
    if eref is not None:
        assert np.array_equal(eout, eref)


def test_two_kinds_of_slots_in_the_serial_order(P):
    """batch = batch_max = 1 (creation indices copied with the leaves)"""
    cfg = W.config("C1")
    kw = dict(batch=1, batch_max=1, max_regions=1 << 14)
    ref, _, st1 = run(P, cfg, slice(0, 1), 4, **kw)
    out, _, st2 = run(P, cfg, slice(0, 1), 4, small_regions=1 << 6, big_share=1e-9, **kw)
    assert st2["regions"] == st1["regions"]
    assert np.array_equal(out, ref)


def test_small_regions_argument_checks(P):
    with pytest.raises(P.PaidError):
        P.Context(small_regions=8)
    with pytest.raises(P.PaidError):
        P.Context(small_regions=1 << 12, big_share=1.5)
