"""The C ABI: the library loads and exports every function include/paid.h
declares (no device needed; no compute call is made)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "paid.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(paid_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("paid_create", "paid_integrate", "paid_destroy", "paid_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paid_1610_09991_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paid_1610_09991_amd import build
        build.build()
    L = P.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(P.EXPORTS) == set(declared_functions())


def test_binding_refuses_to_run_without_the_library(tmp_path, monkeypatch):
    import paid_1610_09991_amd as P
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(RuntimeError):
        P.Context()


def test_create_without_a_device_reports_it():
    """on a host without a GPU the library refuses a context with PAID_EDEVICE
    and a message, and runs nothing on the CPU in its place"""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    import paid_1610_09991_amd as P
    with pytest.raises(P.PaidError) as ei:
        P.Context()
    assert ei.value.code == P.EDEVICE and "device" in str(ei.value)


def test_key_histogram_fixed_point_cannot_overflow():
    """The leaf selection adds keys as fixed-point integers k 2^(62 - ceil(log2 n))
    / maxkey (n leaves, maxkey the largest key), formed as (k 2^-e) * scale with
    e = ilogb(maxkey) so that the scale is finite for every positive finite
    maxkey, subnormal ones included: n keys of at most maxkey, each truncated
    as on the device, sum to at most 2^62 (1 + 2^-50) < 2^63 for every leaf
    count a region code allows (the same arithmetic as the kernel, in Python)."""
    import math
    import sys
    tiny = math.ldexp(1.0, -1074)
    for n in [1, 2, 3, 4, 5, 1000, 2 ** 24, 2 ** 24 + 1, 2 ** 28 - 1, 2 ** 28]:
        lgn = (n - 1).bit_length() if n > 1 else 0
        for maxkey in [tiny, 3 * tiny, 1e-310, 1e-300, 1e-10, 0.3, 1.0, 3.7e5,
                       1e300, sys.float_info.max]:
            e = math.frexp(maxkey)[1] - 1  # ilogb
            scale = math.ldexp(1.0, 62 - lgn) / math.ldexp(maxkey, -e)
            assert math.isfinite(scale), (n, maxkey)
            for k in [maxkey, maxkey * 0.999, maxkey / 3, tiny, 0.0]:
                v = math.ldexp(k, -e) * scale
                assert math.isfinite(v) and v <= math.ldexp(1.0, 62 - lgn) * (1 + 2 ** -50)
            largest = int(math.ldexp(maxkey, -e) * scale)
            assert largest * n <= 2 ** 62 * (1 + 2 ** -50) < 2 ** 63, (n, maxkey)
            # the split leaves the normal-range value unchanged
            if maxkey >= 1e-290 and maxkey <= 1e290:
                assert math.ldexp(maxkey / 3, -e) * scale == \
                    (maxkey / 3) * (math.ldexp(1.0, 62 - lgn) / maxkey), (n, maxkey)



def test_key_bins_stay_a_quarter_octave_wide_below_the_normal_range():
    """The leaf selection bins a key k by the exponent and top two mantissa
    bits of k 2^-e (e = ilogb of the largest key), four bins per octave below
    the largest key.  Scaled this way, keys 2^-j times the largest land in bin
    4j also where k itself is subnormal (raw exponent bits zero), and bins of
    normal keys are those of the unscaled bits (the same arithmetic as the
    kernel, in Python)."""
    import math
    import struct

    def bits(x):
        return struct.unpack("<q", struct.pack("<d", x))[0]

    def key_bin(k, eb):
        if not k > 0.0:
            return 511
        return min(max(eb - (bits(k) >> 50), 0), 511)

    for maxkey in [1e-300, 3e-305, math.ldexp(1.0, -1060), 0.7, 1e300]:
        e = math.frexp(maxkey)[1] - 1
        eb = bits(math.ldexp(maxkey, -e)) >> 50
        for jj in range(0, 127):
            k = math.ldexp(maxkey, -jj)
            if k == 0.0 or math.ldexp(k, jj) != maxkey:
                break  # below the smallest subnormal
            assert key_bin(math.ldexp(k, -e), eb) == 4 * jj, (maxkey, jj)
            if k >= 2.3e-308 and maxkey >= 2.3e-308:
                assert key_bin(k, bits(maxkey) >> 50) == 4 * jj


def test_table_interval_index_needs_no_compare():
    """The frequency-sum table's interval of v = |x| / w: central intervals
    round(8 v) for v < 1, then 8 per octave (9 + 8 floor(log2 v) + the top
    three mantissa bits).  The device forms the central candidate capped at
    8 and the octave candidate from the high word of the double, and takes
    the larger: for v < 1 the octave candidate is never above the central one,
    for v >= 1 it is at least 9.  Checked here against the definition (the
    same arithmetic as the kernel, in Python), negative zero included."""
    import math
    import struct

    def device(x):
        v = abs(x)  # the kernel takes |x| (a negative zero is the interval of 0)
        jc = min(int(math.floor(v * 8 + 0.5)) if v < 2.0 ** 31 else 2 ** 31 - 1, 8)
        hi = struct.unpack("<Q", struct.pack("<d", v))[0] >> 32
        jo = 9 - 1023 * 8 + (hi >> 17)
        return max(jc, jo)

    def definition(x):
        v = abs(x)
        if v < 1.0:
            return int(math.floor(v * 8 + 0.5))
        e = math.frexp(v)[1] - 1  # floor(log2 v)
        m = int(math.floor((v / 2.0 ** e - 1.0) * 8))
        return 9 + 8 * e + m

    vals = [0.0, -0.0, 5e-324, 1e-300, 0.0625, 0.0624999, 0.5, 0.9375, 0.99999999,
            1.0, 1.0000001, 1.125, 1.999999, 2.0, 3.0, 1023.9, 1e6, 1e30]
    vals += [k / 64.0 for k in range(0, 200)]
    vals += [2.0 ** k * (1 + j / 8.0) for k in range(0, 40) for j in range(8)]
    for x in vals:
        assert device(x) == definition(x), x
        assert device(-x) == definition(x), -x


def test_kernel_sign_flips_by_xor_match_the_products():
    """K_j(a, b) flips both energies to x >= 0 (S is odd, S[x,y] = S[-x,-y]):
    the kernel forms x = |a| and y = +-b by XOR of sign bits (the sign of a,
    and of the channel: pp takes -b), where the plain form is f a and f y0
    with f = sign(a) and y0 = b (ph) or -b (pp).  Both agree for every
    nonzero a (a zero a is an even point of S and the two forms differ only
    in the sign of that zero)."""
    import struct

    def bits(v):
        return struct.unpack("<Q", struct.pack("<d", v))[0]

    def dbl(b):
        return struct.unpack("<d", struct.pack("<Q", b))[0]

    SIGN = 1 << 63
    for a in [-3.5, -1e-300, -2.0 ** -1074, 1e-300, 0.25, 7.0, -0.125]:
        for b in [-2.0, -0.0, 0.0, 1e-310, 3.0]:
            for ch in (0, 1):
                sc = 0 if ch else SIGN
                x = abs(a)
                y = dbl(bits(b) ^ (bits(a) & SIGN) ^ sc)
                f = -1.0 if a < 0 else 1.0
                y0 = b if ch else -b
                assert x == f * a and bits(y) == bits(f * y0), (a, b, ch)


def test_node_energies_are_affine_along_a_column():
    """Along a node column the energy -2t (cx + cy) - 4t' cx cy - mu is affine in
    the row's cosine cy: (-2t cx - mu) + cy (-2t - 4t' cx); the kernel forms
    the two coefficients once per column and one FMA per node.  Checked
    against the plain form to rounding over the workloads' parameter ranges."""
    import numpy as np
    rng = np.random.default_rng(5)
    for _ in range(200):
        t, tp, mu = 1.0, rng.uniform(-0.35, 0.0), rng.uniform(-1.2, 0.2)
        cx = rng.uniform(-1, 1)
        cy = rng.uniform(-1, 1, 64)
        plain = -2 * t * (cx + cy) - 4 * tp * cx * cy - mu
        A, B = -2 * t * cx - mu, -2 * t - 4 * tp * cx
        affine = A + cy * B
        scale = 2 * abs(t) * 2 + 4 * abs(tp) + abs(mu)
        assert np.abs(affine - plain).max() <= 8 * np.finfo(float).eps * scale
