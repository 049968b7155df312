"""Lockstep with the serial algorithm: with batch = batch_max = 1 the library
splits, in every round, the leaf of largest key (ties by creation order),
which is the order of the serial Alg. 2 with a max-heap (Listing 2 with
MaxTask = 1).  The final tree must then be the oracle's: the same number of
splits and leaves, the same rectangles, and every leaf's Q_2N the oracle's
rectangle value within the rectangle bar of the parity tests (1e-12 of the
leaf's largest entry: the library's kernel tables are accurate to ~1e-12 of
the local scale; through the C ABI, leaves from paid_set_leaf_output).

Both bubbles are even under p -> -p (the inversion swaps the two energies
and K_j is symmetric in them), so a rectangle and its mirror image have the
same key in exact arithmetic; which of the two is split first is decided by
the last bits of two sums that the two implementations round differently.
The trees are therefore compared up to that choice: leaf by leaf after
mapping each rectangle to the first of itself and its mirror image."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paid_1610_09991_amd as P
    P.lib()
    return P


def canonical(codes):
    """each cell (d, ix, iy) or its mirror image under p -> -p, whichever is first"""
    out = []
    for d, ix, iy in codes:
        m = (d, (1 << d) - 1 - ix, (1 << d) - 1 - iy)
        out.append(min((d, ix, iy), m))
    return sorted(out)


def oracle_codes(rects):
    w = rects[:, 1] - rects[:, 0]
    d = np.round(np.log2(2 * math.pi / w)).astype(int)
    ix = np.round((rects[:, 0] + math.pi) / w).astype(int)
    iy = np.round((rects[:, 2] + math.pi) / w).astype(int)
    return np.stack([d, ix, iy], axis=1)


@pytest.mark.parametrize("ch", ["pp", "ph"])
@pytest.mark.parametrize("layout", [0, 1])
def test_serial_order_leaf_by_leaf(P, ch, layout):
    row = (1.0, -0.25, -0.95, 0.05, 0.3)
    l = (1.07, -2.31)
    rtol = 1e-4
    pch, och = (P.PP, O.PP) if ch == "pp" else (P.PH, O.PH)
    oc = O.Container(W.ff_box(1), 1, t=row[0], tp=row[1], mu=row[2], T=row[3], Omega=row[4],
                     lx=l[0], ly=l[1], channel=och)
    vref, _, sref, rects, qref = oc.integrate_leaves(rtol=rtol, batch=1)
    cap = 4096
    assert len(rects) < cap
    codes = np.zeros((1, cap, 3), dtype=np.int32)
    q2n = np.zeros((1, cap, 45))
    with P.Context(batch=1, batch_max=1, max_regions=cap, eval_layout=layout) as c:
        c.set_leaf_output(codes, q2n)
        out, _, st, rc = c.integrate([row], [l], W.ff_box(1), 1, channels=pch, rtol=rtol)
    assert rc == P.OK
    n = int((codes[0, :, 0] >= 0).sum())
    print(f"{ch} layout {layout}: {n} leaves (oracle {len(rects)}), {st['splits']} splits "
          f"(oracle {sref['splits']})")
    assert n == len(rects) and st["splits"] == sref["splits"]
    # the same rectangles, up to the choice between mirror images
    gcodes = codes[0, :n]
    assert canonical(map(tuple, gcodes)) == canonical(map(tuple, oracle_codes(rects)))
    # Q_2N of every leaf against the oracle's rule on the same rectangle
    dev = 0.0
    for (d, ix, iy), g in zip(gcodes, q2n[0, :n]):
        w = 2 * math.pi / 2 ** d
        x0, y0 = -math.pi + ix * w, -math.pi + iy * w
        _, ref = oc.region(x0, x0 + w, y0, y0 + w)
        dev = max(dev, float(np.abs(g - ref).max() / np.abs(ref).max()))
    print(f"worst leaf deviation {dev:.2e} of the leaf's largest entry")
    assert dev <= 1e-12
    # the values: sums of the same leaves (exactly when no mirror choice
    # differs), else within the tolerance
    scale = np.maximum(np.abs(vref), 1e-3 * np.abs(vref).max())
    assert (np.abs(out[0, 0, 0] - vref) <= rtol * scale).all()
