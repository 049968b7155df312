"""GPU parity: libpaid (HIP, gfx950) against the FP64 CPU oracle, through the
C ABI.  Gate for floating point (per integral, same seeded inputs):
    |gpu_pq - ref_pq| <= rtol * max(|ref_pq|, nu * max |ref|),  nu = 1e-3,
with ref the oracle at rtol/1000.  Kernel and rectangle values are compared
element by element at rounding level."""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

NU = 1e-3
THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def P():
    import paid_1610_09991_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module", params=["separable", "mfma"])
def ctx(P, request):
    gram = P.GRAM_SEPARABLE if request.param == "separable" else P.GRAM_MFMA
    c = P.Context(max_regions=1 << 16, max_active=512, gram=gram)  # FP64 either way
    yield c
    c.close()


def gate_ratio(gpu, ref, rtol):
    scale = np.maximum(np.abs(ref), NU * np.abs(ref).max())
    return float((np.abs(gpu - ref) / (rtol * scale)).max())


def oracle_refs(cfg, picks, rtol):
    """oracle values for (param index, q index, channel) picks"""
    conts = []
    for ip, iq, ch in picks:
        p = cfg["params"][ip]
        conts.append(O.Container(cfg["ff"], cfg["L"], t=p[0], tp=p[1], mu=p[2], T=p[3],
                                 Omega=p[4], lx=cfg["q"][iq][0], ly=cfg["q"][iq][1],
                                 channel=ch))
    vals, _, _, nc = O.integrate_batch(conts, rtol=rtol, err_mode=O.ERR_GLOBAL, batch=4,
                                       nthreads=THREADS)
    assert nc == 0
    return vals


# ------------------------------------------------------------------ kernel
def adversarial(Om, T, emax):
    pts = []
    for k in (1, 3, 6, 9, 12, 15):
        d = 10.0 ** -k
        pts += [(Om * (1 + d), Om * (1 - d)), (Om * (1 + d), -Om), (-Om * (1 - d), Om),
                (0.37 * (1 + d), 0.37), (0.37 * (1 + d), -0.37), (d * T, -2 * d * T),
                (-1.3 * (1 + d), -1.3), (3.1, 3.1 * (1 - d))]
    pts += [(0.0, 0.0), (emax * 0.999, -emax * 0.999), (emax * 0.999, emax * 0.998)]
    rng = np.random.default_rng(7)
    pts += [tuple(x) for x in rng.uniform(-emax * 0.99, emax * 0.99, (40, 2))]
    return [(a, b) for a, b in pts if abs(a) <= emax and abs(b) <= emax]


@pytest.mark.parametrize("T,Om", [(0.005, 0.01), (0.01, 0.1), (0.1, 1.0), (0.01, 10.0),
                                  (0.05, 0.0)])
def test_kernel_matches_oracle_at_rounding_level(ctx, P, T, Om):
    row = (1.0, -0.25, -0.95, T, Om)
    emax = 4 + 1 + 0.95
    pts = adversarial(max(Om, 1e-3), T, emax)
    a = np.array([p[0] for p in pts])
    b = np.array([p[1] for p in pts])
    for ch, och in ((P.PH, O.PH), (P.PP, O.PP)):
        g = ctx.kernel(row, a, b, ch)
        for x, y, v in zip(a, b, g):
            ref = O.kernel(x, y, Om, T, och)
            loc = abs(O.kernel(abs(x) + 0.5 * T, abs(x) + 0.5 * T, Om, T, O.PH))
            assert abs(v - ref) <= 2e-12 * max(abs(ref), loc), (ch, x, y, v, ref)


def test_kernel_rejects_energies_outside_the_band(ctx, P):
    with pytest.raises(P.PaidError):
        ctx.kernel((1.0, 0.0, 0.0, 0.1, 0.1), [4.5], [0.0])


# ------------------------------------------------------------------ rectangles
@pytest.mark.parametrize("ff_name", ["ff9", "ff5", "ff25", "ff1"])
@pytest.mark.parametrize("ch", ["pp", "ph"])
def test_children_match_oracle_rectangles(ctx, P, ff_name, ch):
    ff, L = {"ff9": (W.ff_box(1), 1), "ff5": (W.ff5(), 1), "ff25": (W.ff_box(2), 2),
             "ff1": (W.ff_box(0), 0)}[ff_name]
    pch, och = (P.PP, O.PP) if ch == "pp" else (P.PH, O.PH)
    row = (1.0, -0.3, -1.1, 0.02, 0.05)
    l = (2.88, 0.26)
    rng = np.random.default_rng(3)
    codes = [(0, 0, 0), (1, 1, 0), (2, 3, 1)]
    for d in (4, 7, 11):
        for _ in range(3):
            codes.append((d, int(rng.integers(0, 2 ** d)), int(rng.integers(0, 2 ** d))))
    codes = np.array(codes)
    q2n, keys = ctx.children(row, l, pch, ff, L, codes)
    c = O.Container(ff, L, t=row[0], tp=row[1], mu=row[2], T=row[3], Omega=row[4], lx=l[0],
                    ly=l[1], channel=och)
    for i, (d, ix, iy) in enumerate(codes):
        w = 2 * math.pi / 2 ** d
        for k in range(4):
            cx, cy = k & 1, k >> 1
            x0 = -math.pi + ix * w + cx * w / 2
            y0 = -math.pi + iy * w + cy * w / 2
            qn, ref = c.region(x0, x0 + w / 2, y0, y0 + w / 2)
            big = np.abs(ref).max() + 1e-300
            assert np.abs(q2n[i, k] - ref).max() <= 1e-12 * big, (i, k)
            # error of the pair: same quantity, different rounding order
            ek = np.abs(qn - ref).sum()
            assert abs(keys[i, k] - ek) <= 1e-12 * np.abs(ref).sum() + 1e-7 * ek, (i, k)


def _children_against_oracle(c, P, row, l, ff, L, codes, tol=1e-12):
    q2n, keys = c.children(row, l, P.PH, ff, L, codes)
    oc = O.Container(ff, L, t=row[0], tp=row[1], mu=row[2], T=row[3], Omega=row[4], lx=l[0],
                     ly=l[1], channel=O.PH)
    for i, (d, ix, iy) in enumerate(codes):
        w = 2 * math.pi / 2 ** d
        for k in range(4):
            x0 = -math.pi + ix * w + (k & 1) * w / 2
            y0 = -math.pi + iy * w + (k >> 1) * w / 2
            qn, ref = oc.region(x0, x0 + w / 2, y0, y0 + w / 2)
            assert np.abs(q2n[i, k] - ref).max() <= tol * np.abs(ref).max(), (row, i, k)


def test_children_with_a_long_frequency_table(ctx, P):
    """T = 1e-4 against a band of 6.3: a table of 129 rows, staged whole in LDS"""
    codes = np.array([(0, 0, 0), (5, 7, 20), (9, 300, 100)])
    _children_against_oracle(ctx, P, (1.0, -0.3, -1.1, 1e-4, 0.05), (2.88, 0.26), W.ff_box(1), 1,
                             codes)


def test_children_with_a_table_past_64k_of_lds(P):
    """T = 1.5e-6: 177 table rows (25.5 KB) beside the per-wave scratch of a
    general 25-function set (38.6 KB) exceed 64 KiB; the workgroup then takes
    one wave and the device's LDS limit.  On a device with more than 64 KiB
    per workgroup (gfx950: 160 KiB) the rectangles must be computed and match
    the oracle; elsewhere the call is refused with a clear error."""
    import torch
    props = torch.cuda.get_device_properties(0)
    limit = max(getattr(props, "shared_memory_per_block_optin", 0),
                getattr(props, "shared_memory_per_block", 0))
    print(f"{props.gcnArchName}: {limit} bytes of LDS per workgroup")
    rng = np.random.default_rng(11)
    ff = np.linalg.qr(rng.normal(size=(25, 25)))[0][:6]  # 6 orthonormal rows, not the box
    codes = np.array([(6, 40, 17)])
    row, l = (1.0, -0.3, -1.1, 1.5e-6, 0.05), (2.88, 0.26)
    with P.Context() as c:
        if limit > 65536:
            _children_against_oracle(c, P, row, l, ff, 2, codes)
        else:
            with pytest.raises(P.PaidError) as ei:
                _children_against_oracle(c, P, row, l, ff, 2, codes)
            assert "does not fit in LDS" in str(ei.value)


# ------------------------------------------------------------------ full integrations
def test_c1_full_workload(ctx, P):
    """8x8 q, FF5, pp+ph at the workload's rtol 1e-4 and at 1e-6."""
    cfg = W.config("C1")
    picks = W.containers(cfg)
    ref = oracle_refs(cfg, picks, 1e-10)
    for rtol in (1e-4, 1e-6):
        out, _, st, rc = ctx.integrate(cfg["params"], cfg["q"], cfg["ff"], cfg["L"], rtol=rtol)
        assert rc == P.OK and st["not_converged"] == 0
        for k, (ip, iq, ch) in enumerate(picks):
            assert gate_ratio(out[ip, iq, ch], ref[k], rtol) <= 1.0, (rtol, ip, iq, ch)
            assert np.array_equal(out[ip, iq, ch], out[ip, iq, ch].T)


def test_batched_random_parameter_sets(ctx, P):
    """Uneven refinement depths in one call: random (mu, T, t', Omega) rows."""
    p = W.random_params(6, seed=3, omega_range=(0.05, 1.0))
    p[:, 3] = np.maximum(p[:, 3], 0.02)  # keep the oracle reference quick
    q = W.q_grid(16)[[0, 17, 100, 255]]
    cfg = dict(params=p, q=q, ff=W.ff_box(1), L=1, channels=3)
    out, e, st, rc = ctx.integrate(p, q, cfg["ff"], 1, rtol=1e-6, err=True)
    assert rc == P.OK
    picks = W.containers(cfg)
    ref = oracle_refs(cfg, picks, 1e-9)
    for k, (ip, iq, ch) in enumerate(picks):
        assert gate_ratio(out[ip, iq, ch], ref[k], 1e-6) <= 1.0, (ip, iq, ch)
        assert (e[ip, iq, ch] >= 0).all()


@pytest.mark.parametrize("ch", [1, 2, 3])
def test_channel_subsets_and_edge_momenta(ctx, P, ch):
    p = np.array([[1.0, -0.25, -0.95, 0.05, 0.2]])
    q = np.array([[math.pi, math.pi], [-math.pi, 0.0], [0.0, 0.0], [7.5, -13.0], [1.0, 2.0]])
    out, _, st, rc = ctx.integrate(p, q, W.ff_box(1), 1, channels=ch, rtol=1e-7)
    assert rc == P.OK and out.shape == (1, 5, 1 if ch < 3 else 2, 9, 9)
    chans = [c for c, bit in ((O.PP, 1), (O.PH, 2)) if ch & bit]
    cfg = dict(params=p, q=q, ff=W.ff_box(1), L=1, channels=ch)
    ref = oracle_refs(cfg, W.containers(cfg), 1e-10)
    for k, (ip, iq, c) in enumerate(W.containers(cfg)):
        assert gate_ratio(out[ip, iq, chans.index(c)], ref[k], 1e-7) <= 1.0


@pytest.mark.parametrize("ff_name", ["ff5", "ff25", "ff1"])
def test_form_factor_sets(ctx, P, ff_name):
    ff, L = {"ff5": (W.ff5(), 1), "ff25": (W.ff_box(2), 2), "ff1": (W.ff_box(0), 0)}[ff_name]
    p = np.array([[1.0, -0.3, -1.1, 0.05, 0.3]])
    q = np.array([[2.88, 0.26], [0.0, 0.0]])
    out, _, st, rc = ctx.integrate(p, q, ff, L, rtol=1e-6)
    assert rc == P.OK
    cfg = dict(params=p, q=q, ff=ff, L=L, channels=3)
    ref = oracle_refs(cfg, W.containers(cfg), 1e-9)
    for k, (ip, iq, c) in enumerate(W.containers(cfg)):
        assert gate_ratio(out[ip, iq, c], ref[k], 1e-6) <= 1.0


def test_unit_and_gaussian_integrands(P):
    with P.Context(kind=P.UNIT, max_regions=1 << 16) as c:
        out, _, _, rc = c.integrate([[1, 0, 0, 0.1, 0.1]], [[0.3, 0.2]], W.ff_box(2), 2,
                                    rtol=1e-10, atol=1e-12)
        assert rc == P.OK
        assert np.abs(out[0, 0, 0] - np.eye(25)).max() < 1e-10
    x0, y0, s = 0.7, -2.9, 0.15
    with P.Context(kind=P.GAUSS, gauss=(x0, y0, s), max_regions=1 << 14) as c:
        out, e, _, rc = c.integrate([[1, 0, 0, 0.1, 0.1]], [[0.0, 0.0]], W.ff_box(0), 0,
                                    channels=P.PH, rtol=1e-10, err=True)
        from scipy import special
        f = lambda cc: special.ndtr((math.pi - cc) / s) - special.ndtr((-math.pi - cc) / s)
        exact = 2 * math.pi * s * s * f(x0) * f(y0) / (4 * math.pi ** 2)
        assert abs(out[0, 0, 0, 0, 0] - exact) <= 1e-10 * exact
        assert abs(out[0, 0, 0, 0, 0] - exact) <= e[0, 0, 0, 0, 0] + 1e-16


def test_integrand_at_the_bottom_of_the_double_range(P):
    """A wide Gaussian centred 37 widths outside the zone: values ~1e-297,
    integral ~2e-299, leaf errors (the keys of the leaf selection) far below
    ~2.6e-290, where 2^62 / (largest key) is not a finite double.  The global
    mode still meets rtol 1e-10 against the closed form; the per-integral mode,
    whose per-leaf errors are FP32, must end ENOCONV (its tolerance ~2e-309 is
    below FP32's range) instead of passing on errors rounded to zero."""
    from scipy import special
    x0, y0, s = math.pi + 370.0, 0.0, 10.0
    f = lambda cc: special.ndtr((math.pi - cc) / s) - special.ndtr((-math.pi - cc) / s)
    exact = 2 * math.pi * s * s * f(x0) * f(y0) / (4 * math.pi ** 2)
    assert 1e-300 < exact < 1e-298
    args = ([[1, 0, 0, 0.1, 0.1]], [[0.0, 0.0]], W.ff_box(0), 0)
    with P.Context(kind=P.GAUSS, gauss=(x0, y0, s), max_regions=1 << 14) as c:
        out, e, st, rc = c.integrate(*args, channels=P.PH, rtol=1e-10, err=True)
    print("global", rc, st, out[0, 0, 0, 0, 0], exact, flush=True)
    assert rc == P.OK
    assert abs(out[0, 0, 0, 0, 0] - exact) <= 1e-10 * exact
    assert abs(out[0, 0, 0, 0, 0] - exact) <= e[0, 0, 0, 0, 0] + 1e-310
    with P.Context(kind=P.GAUSS, gauss=(x0, y0, s), err_mode=P.ERR_PER_INTEGRAL,
                   max_regions=1 << 10) as c:
        out, e, st, rc = c.integrate(*args, channels=P.PH, rtol=1e-10, err=True)
    print("per integral", rc, st, flush=True)
    assert rc == P.ENOCONV and st["not_converged"] == 1
    assert np.isfinite(out).all()


def test_per_integral_mode(P):
    p = np.array([[1.0, -0.25, -0.95, 0.05, 0.2]])
    q = np.array([[1.57, 1.31]])
    with P.Context(err_mode=P.ERR_PER_INTEGRAL, max_regions=1 << 17) as c:
        out, e, st, rc = c.integrate(p, q, W.ff_box(1), 1, rtol=1e-6, err=True)
    assert rc == P.OK
    tau = 1e-6 * np.maximum(np.abs(out), NU * np.abs(out).max(axis=(-1, -2), keepdims=True))
    assert (e <= tau * (1 + 1e-9)).all()
    cfg = dict(params=p, q=q, ff=W.ff_box(1), L=1, channels=3)
    ref = oracle_refs(cfg, W.containers(cfg), 1e-10)
    for k, (ip, iq, c) in enumerate(W.containers(cfg)):
        assert gate_ratio(out[ip, iq, c], ref[k], 1e-6) <= 1.0


def test_budget_exhaustion_reports_noconv(P):
    with P.Context(max_regions=64) as c:
        out, e, st, rc = c.integrate([[1.0, -0.25, -0.95, 0.01, 0.01]], [[1.0, 0.5]],
                                     W.ff_box(1), 1, rtol=1e-9, err=True)
    assert rc == P.ENOCONV and st["not_converged"] == 2
    assert np.isfinite(out).all() and (e > 0).any()


def test_refinement_stops_at_the_deepest_code(P):
    """A Gaussian of width 1e-10 centred on a corner that every level keeps
    as a node: the error estimate never drops below the tolerance before the
    rectangles reach the smallest side a region code holds (2 pi / 2^28);
    the container then stops with the budget flag (ENOCONV) instead of
    splitting further (at most four splits per round, so that the region
    budget is not what stops it)."""
    with P.Context(kind=P.GAUSS, gauss=(0.0, 0.0, 1e-10), max_regions=1 << 14, batch=1,
                   batch_max=4) as c:
        out, e, st, rc = c.integrate([[1, 0, 0, 0.1, 0.1]], [[0.0, 0.0]], W.ff_box(0), 0,
                                     channels=P.PH, rtol=1e-8, err=True)
    assert rc == P.ENOCONV and st["not_converged"] == 1
    assert st["max_depth"] == 28 and st["regions"] < (1 << 14)
    assert np.isfinite(out).all() and np.isfinite(e).all()


def test_results_are_bitwise_reproducible(ctx, P):
    cfg = W.config("C1")
    a, _, _, _ = ctx.integrate(cfg["params"], cfg["q"][:20], cfg["ff"], 1, rtol=1e-6)
    b, _, _, _ = ctx.integrate(cfg["params"], cfg["q"][:20], cfg["ff"], 1, rtol=1e-6)
    assert np.array_equal(a, b)


def test_invalid_arguments_are_rejected(ctx, P):
    p = [[1.0, 0.0, 0.0, 0.1, 0.1]]
    bad = [dict(ff=np.ones((2, 9)), L=1), dict(ff=W.ff_box(1), L=3),
           dict(ff=W.ff_box(1), L=1, channels=0), dict(ff=W.ff_box(1), L=1, rtol=0.0),
           dict(ff=W.ff_box(1), L=1, params=[[1.0, 0.0, 0.0, 0.0, 0.1]])]
    for b in bad:
        with pytest.raises(P.PaidError) as ei:
            ctx.integrate(b.get("params", p), [[0.1, 0.2]], b["ff"], b["L"],
                          channels=b.get("channels", 3), rtol=b.get("rtol", 1e-6))
        assert ei.value.code == P.EINVAL


def test_empty_inputs(ctx, P):
    """an empty batch is refused (EINVAL); an empty list of energies or of
    transfer momenta to contract gives empty results"""
    p = [[1.0, -0.25, -0.95, 0.05, 0.1]]
    for params, q in ((p, np.zeros((0, 2))), (np.zeros((0, 5)), [[0.1, 0.2]])):
        with pytest.raises(P.PaidError) as ei:
            ctx.integrate(params, q, W.ff_box(1), 1)
        assert ei.value.code == P.EINVAL
    with pytest.raises(P.PaidError) as ei:
        ctx.children(p[0], (0.1, 0.2), P.PH, W.ff_box(1), 1, np.zeros((0, 3), dtype=np.int32))
    assert ei.value.code == P.EINVAL
    assert ctx.kernel(p[0], [], []).shape == (0,)
    z = np.zeros((0, 9, 9))
    dP, dC, dD = ctx.contract(np.zeros((0, 2, 9, 9)), z, z, z)
    assert dP.shape == dC.shape == dD.shape == (0, 9, 9)


def test_full_size_workload_sampled(P):
    """The benchmark's workload at full size (23,040 containers, one call) in
    the benchmark's launch configuration (graph-replayed rounds, the shipped
    launch profile), plain and with the shipped seed model; sampled
    containers against the oracle."""
    import json
    import os
    from paid_1610_09991_amd import seed_model as SM
    cfg = W.config("C2")
    here = os.path.dirname(P.__file__)
    with open(os.path.join(here, "tuned_c2.json")) as f:
        tuned = json.load(f)["config"]
    w, meta = SM.load()
    c = P.Context(graph=1, **tuned)
    runs = {}
    for name, model in (("plain", None), ("seeded", w)):
        c.set_seed_model(model, kappa=meta["kappa"])
        out, _, st, rc = c.integrate(cfg["params"], cfg["q"], cfg["ff"], cfg["L"], rtol=1e-6)
        assert rc == P.OK and st["not_converged"] == 0 and np.isfinite(out).all(), name
        assert (st["seeded"] > 0) == (model is not None)
        runs[name] = out
    c.close()
    rng = np.random.default_rng(5)
    picks = [(ip, int(rng.integers(0, 576)), int(rng.integers(0, 2))) for ip in (0, 5, 9, 12, 14)]
    ref = oracle_refs(cfg, picks, 1e-9)
    for name, out in runs.items():
        for k, (ip, iq, ch) in enumerate(picks):
            assert gate_ratio(out[ip, iq, ch], ref[k], 1e-6) <= 1.0, (name, ip, iq, ch)
        # symmetry of every output matrix
        assert np.array_equal(out, np.swapaxes(out, -1, -2))


# ------------------------------------------------------------------ half-zone mode
@pytest.mark.parametrize("gram", ["separable", "mfma"])
def test_half_zone_mode_matches_the_oracle(P, gram):
    """symmetry = 1 integrates p_y >= 0 only and weights each box pair by its
    parity (0 or 2).  On C1 (FF5: s, extended s, d and the two p-waves, which
    are odd) every integral is within the gate of the full-zone oracle, the
    pairs of odd joint parity are exactly zero, and the trees hold about half
    the leaves of the full-zone run."""
    cfg = W.config("C1")
    picks = W.containers(cfg)
    ref = oracle_refs(cfg, picks, 1e-10)
    g = P.GRAM_SEPARABLE if gram == "separable" else P.GRAM_MFMA
    res = {}
    for sym in (0, 1):
        with P.Context(max_regions=1 << 16, max_active=512, gram=g, symmetry=sym) as c:
            res[sym] = c.integrate(cfg["params"], cfg["q"], cfg["ff"], cfg["L"], rtol=1e-6)
    out, _, st, rc = res[1]
    assert rc == P.OK and st["not_converged"] == 0
    for k, (ip, iq, ch) in enumerate(picks):
        assert gate_ratio(out[ip, iq, ch], ref[k], 1e-6) <= 1.0, (ip, iq, ch)
    assert np.all(out[..., :3, 3:] == 0.0) and np.all(out[..., 3:, :3] == 0.0)
    assert np.array_equal(out, np.swapaxes(out, -1, -2))
    print(f"half zone: {st['regions']} leaves against {res[0][2]['regions']} on the full zone")
    assert st["regions"] < 0.6 * res[0][2]["regions"]


@pytest.mark.parametrize("mode", ["per_integral", "weighted"])
def test_half_zone_mode_with_other_error_tests(P, mode):
    """the half-zone mode under the per-integral and the weighted tests, with
    the 25-function box set (odd pairs: one of the two functions has an odd
    number of sine factors)"""
    row = [1.0, -0.25, -0.95, 0.05, 0.2]
    q = np.array([[2.88, 0.26], [1.57, 1.31], [0.0, 0.0]])
    ff, L = W.ff_box(2), 2
    cfg = dict(params=np.array([row]), q=q, ff=ff, L=L)
    picks = [(0, iq, ch) for iq in range(3) for ch in (O.PP, O.PH)]
    ref = oracle_refs(cfg, picks, 1e-9)
    em = P.ERR_PER_INTEGRAL if mode == "per_integral" else P.ERR_WEIGHTED
    with P.Context(max_regions=1 << 16, err_mode=em, symmetry=1) as c:
        if mode == "weighted":
            # w_pp = 1, w_pq = 1/2: the global test's weights
            c.set_pair_weights(np.broadcast_to(np.full((25, 25), 0.5) + 0.5 * np.eye(25),
                                               (6, 25, 25)).copy())
        out, _, st, rc = c.integrate([row], q, ff, L, rtol=1e-6)
    assert rc == P.OK and st["not_converged"] == 0
    odd = np.array([(((a // 5) in (2, 4)) ^ ((a % 5) in (2, 4))) for a in range(25)])
    mask = odd[:, None] ^ odd[None, :]
    for k, (ip, iq, ch) in enumerate(picks):
        assert gate_ratio(out[ip, iq, ch], ref[k], 1e-6) <= 1.0, (iq, ch)
        assert np.all(out[ip, iq, ch][mask] == 0.0)


def test_half_zone_mode_argument_checks(P):
    with pytest.raises(P.PaidError):
        P.Context(symmetry=2)
    with pytest.raises(P.PaidError):
        P.Context(kind=P.GAUSS, symmetry=1)
    from paid_1610_09991_amd import seed_model as SM
    w, meta = SM.load()
    with P.Context(symmetry=1) as c:
        c.set_seed_model(w, kappa=meta["kappa"])
        with pytest.raises(P.PaidError):
            c.integrate([[1.0, -0.25, -0.95, 0.05, 0.2]], [[0.3, 0.2]], W.ff_box(1), 1)


# ------------------------------------------------------------------ reduced precision
# The dense Gram in FP32 or with three-term bf16 splits (FP32 accumulation)
# carries ~2^-24 relative error per product; region sums, the error estimate
# and the termination test stay FP64.  Stated tolerance of these modes: every
# rectangle within 2e-6 of its largest entry, every integral within the gate
# at rtol 2e-5 (observed values are printed).
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("ff_name", ["ff9", "ff25"])
def test_reduced_precision_rectangles(P, prec, ff_name):
    ff, L = (W.ff_box(1), 1) if ff_name == "ff9" else (W.ff_box(2), 2)
    pr = P.FP32 if prec == "fp32" else P.BF16X3
    row = (1.0, -0.3, -1.1, 0.02, 0.05)
    l = (2.88, 0.26)
    codes = np.array([(0, 0, 0), (2, 1, 3), (6, 17, 40), (10, 700, 12)])
    with P.Context(gram=P.GRAM_MFMA, precision=pr) as c:
        q2n, keys = c.children(row, l, P.PH, ff, L, codes)
    oc = O.Container(ff, L, t=row[0], tp=row[1], mu=row[2], T=row[3], Omega=row[4], lx=l[0],
                     ly=l[1], channel=O.PH)
    worst = 0.0
    for i, (d, ix, iy) in enumerate(codes):
        w = 2 * math.pi / 2 ** d
        for k in range(4):
            x0 = -math.pi + ix * w + (k & 1) * w / 2
            y0 = -math.pi + iy * w + (k >> 1) * w / 2
            qn, ref = oc.region(x0, x0 + w / 2, y0, y0 + w / 2)
            worst = max(worst, np.abs(q2n[i, k] - ref).max() / np.abs(ref).max())
    print(f"{prec} {ff_name}: worst rectangle error {worst:.2e} of the largest entry")
    assert worst <= 2e-6


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_reduced_precision_integrals(P, prec):
    pr = P.FP32 if prec == "fp32" else P.BF16X3
    p = np.array([[1.0, -0.3, -1.1, 0.05, 0.3]])
    q = np.array([[2.88, 0.26], [0.0, 0.0], [1.0, -2.0]])
    ff, L = W.ff_box(2), 2
    with P.Context(gram=P.GRAM_MFMA, precision=pr, max_regions=1 << 16) as c:
        out, _, st, rc = c.integrate(p, q, ff, L, rtol=1e-6)
    assert rc == P.OK
    cfg = dict(params=p, q=q, ff=ff, L=L, channels=3)
    ref = oracle_refs(cfg, W.containers(cfg), 1e-9)
    worst = max(gate_ratio(out[ip, iq, c], ref[k], 1.0)
                for k, (ip, iq, c) in enumerate(W.containers(cfg)))
    print(f"{prec}: worst integral error {worst:.2e} (gate units of rtol = 1)")
    assert worst <= 2e-5


def test_graph_replayed_rounds_match_eager_rounds(P):
    """Rounds replayed from one captured HIP graph give bit-identical results
    and statistics to rounds launched one kernel at a time, call after call,
    with other work on the device in between (fewer slots than containers,
    so admission runs in many rounds)."""
    cfg = W.config("C1")
    args = (cfg["params"], cfg["q"], cfg["ff"], cfg["L"])
    with P.Context(max_regions=1 << 14, max_active=24) as eager, \
            P.Context(max_regions=1 << 14, max_active=24, graph=1) as graph:
        ref, eref, sref, _ = eager.integrate(*args, rtol=1e-5, err=True)
        for rep in range(3):
            got, egot, sgot, _ = graph.integrate(*args, rtol=1e-5, err=True)
            assert np.array_equal(got, ref) and np.array_equal(egot, eref), rep
            for k in ("regions", "splits", "kernel_evals", "rounds", "launch_rounds"):
                assert sgot[k] == sref[k], (rep, k)
            eager.integrate(cfg["params"], cfg["q"][:5], cfg["ff"], cfg["L"], rtol=1e-4)


# ------------------------------------------------------------------ weighted global test
def test_weighted_mode_with_unit_pair_weights_is_the_global_mode(P):
    cfg = W.config("C1")
    n = len(cfg["q"]) * 2
    Wm = np.broadcast_to(np.full((5, 5), 0.5) + 0.5 * np.eye(5), (n, 5, 5)).copy()
    args = (cfg["params"], cfg["q"], cfg["ff"], cfg["L"])
    with P.Context(max_regions=1 << 14, max_active=64) as g, \
            P.Context(max_regions=1 << 14, max_active=64, err_mode=P.ERR_WEIGHTED) as w:
        a, _, sa, _ = g.integrate(*args, rtol=1e-6)
        w.set_pair_weights(Wm)
        b, _, sb, _ = w.integrate(*args, rtol=1e-6)
    assert np.array_equal(a, b) and sa["regions"] == sb["regions"]


def test_weighted_mode_bounds_the_contracted_error(P):
    """weights from random couplings per container (Eq. P_globerr read as a
    bound of the contracted matrices' summed error): the weighted error of
    every container against the oracle stays within rtol of its weighted sum"""
    cfg = W.config("C1")
    q = cfg["q"][[2, 19, 33, 50]]
    p = cfg["params"][0]
    rng = np.random.default_rng(12)
    Ws = np.stack([O.weights_from_couplings(rng.normal(size=(5, 5))) for _ in range(len(q) * 2)])
    with P.Context(max_regions=1 << 15, max_active=16, err_mode=P.ERR_WEIGHTED) as w:
        w.set_pair_weights(Ws)
        out, _, st, rc = w.integrate(cfg["params"], q, cfg["ff"], cfg["L"], rtol=1e-6)
    assert rc == 0
    conts = [O.Container(cfg["ff"], cfg["L"], t=p[0], tp=p[1], mu=p[2], T=p[3], Omega=p[4],
                         lx=l[0], ly=l[1], channel=ch) for l in q for ch in (O.PP, O.PH)]
    ref, _, _, nc = O.integrate_batch(conts, rtol=1e-10, err_mode=O.ERR_GLOBAL, batch=4,
                                      nthreads=THREADS)
    assert nc == 0
    gpu = out.reshape(-1, 5, 5)
    iu = np.triu_indices(5)
    for k in range(len(conts)):
        pw = np.where(np.eye(5) > 0, Ws[k], Ws[k] + Ws[k].T)[iu]
        err = np.sum(pw * np.abs(gpu[k][iu] - ref[k][iu]))
        assert err <= 1e-6 * np.sum(pw * np.abs(ref[k][iu])), k


def test_weighted_mode_argument_checks(P):
    cfg = W.config("C1")
    with P.Context(err_mode=P.ERR_WEIGHTED) as w:
        with pytest.raises(P.PaidError):  # no weights set
            w.integrate(cfg["params"], cfg["q"][:1], cfg["ff"], cfg["L"], rtol=1e-4)
        bad = np.ones((2, 5, 5))
        bad[1, 2, 3] = -1.0
        w.set_pair_weights(bad)
        with pytest.raises(P.PaidError):
            w.integrate(cfg["params"], cfg["q"][:1], cfg["ff"], cfg["L"], rtol=1e-4)
