"""Pins of the oracle's stochastic rounding (storage formats bf16sr, fp16sr),
CPU only.

A stochastically rounded value is one of the two grid points that bracket
it, chosen with the 8 low bits u8 of the site's Philox word so that, over the
256 values of u8, it lands on the upper one in the nearest whole number of
cases to 256 f (f the value's distance from the lower point in grid
spacings): the mean of the 256 results is the value itself up to 1/512 of a
spacing.  The brackets here come from numpy's own float16 and from float32
bit patterns (BF16 is the upper half of an FP32 word), not from the oracle's
grid arithmetic."""

import numpy as np
import pytest

import oracle as orc

U8 = np.arange(256)


def _bracket_bf16(v):
    """Grid points of BF16 below and above |v|: |v| toward zero to FP32, then
    the low 16 bits of that word cleared (every BF16 value is an FP32 one)."""
    a = np.float32(abs(float(v)))
    if float(a) > abs(float(v)):
        a = np.nextafter(a, np.float32(0))
    b = int(np.array([a], dtype=np.float32).view(np.uint32)[0])
    lo = np.array([b & 0xFFFF0000], dtype=np.uint32).view(np.float32)[0]
    hi = np.array([(b & 0xFFFF0000) + 0x10000], dtype=np.uint32).view(np.float32)[0]
    return float(lo), float(hi)


def _bracket_f16(v):
    a = abs(float(v))
    n = np.float16(a)
    if float(n) > a:
        n = np.nextafter(n, np.float16(0))
    return float(n), float(np.nextafter(n, np.float16(np.inf)))


def _values(rng, n):
    v = rng.standard_normal(n).astype(np.float32) * np.float32(0.7)
    return v[v != 0]


@pytest.mark.parametrize("storage,bracket", [("bf16sr", _bracket_bf16), ("fp16sr", _bracket_f16)])
def test_result_is_a_bracketing_grid_point_and_unbiased(storage, bracket):
    rng = np.random.default_rng(3)
    vals = list(_values(rng, 60))
    if storage == "fp16sr":  # FP16's subnormal grid (spacing 2^-24) and its smallest normals
        vals += [3.3 * 2.0 ** -24, -7.77 * 2.0 ** -22, 2.0 ** -14 * 1.0003, 1e-9]
    for v in vals:
        lo, hi = bracket(v)
        s = np.sign(v)
        got = np.array([orc.round_storage(float(v), storage, u) for u in U8])
        assert np.all((got == s * lo) | (got == s * hi)), (v, lo, hi)
        ups = got == s * hi
        # the rounding-up draws are the top ones (u8 >= some threshold)
        k = int(ups.sum())
        assert np.all(ups[256 - k:]) and not np.any(ups[: 256 - k]), v
        # and their number is the nearest integer to 256 f: mean = v to 1/512 of the spacing
        f = (abs(float(v)) - lo) / (hi - lo)
        assert abs(k - 256 * f) <= 0.5 + 1e-9, (v, k, 256 * f)
        assert abs(got.mean() - float(v)) <= (hi - lo) / 512 * (1 + 1e-9)


@pytest.mark.parametrize("storage", ["bf16sr", "fp16sr"])
def test_grid_values_are_kept_and_sign_is_symmetric(storage):
    grid = [1.0, -0.75, 2.0 ** -9, 1.0078125, 3.0 * 2.0 ** -24 if storage == "fp16sr" else 3.0 * 2.0 ** -130]
    for g in grid:
        assert all(orc.round_storage(g, storage, u) == g for u in U8), g
    rng = np.random.default_rng(5)
    for v in _values(rng, 20):
        for u in (0, 77, 128, 255):
            assert orc.round_storage(-float(v), storage, u) == -orc.round_storage(float(v), storage, u)


def test_worked_examples():
    # BF16 spacing at 1 is 2^-7; 1 + 0.3 * 2^-7 sits 0.3 spacings above 1:
    # up when u8 >= 255.5 - 76.8 = 178.7, i.e. for u8 = 179 .. 255 (77 of 256)
    v = 1.0 + 0.3 * 2.0 ** -7
    assert orc.round_storage(v, "bf16sr", 178) == 1.0
    assert orc.round_storage(v, "bf16sr", 179) == 1.0 + 2.0 ** -7
    # FP16 subnormal grid: 3.3 * 2^-24 rounds to 3 or 4 * 2^-24, the same way
    w = 3.3 * 2.0 ** -24
    assert orc.round_storage(w, "fp16sr", 178) == 3.0 * 2.0 ** -24
    assert orc.round_storage(w, "fp16sr", 179) == 4.0 * 2.0 ** -24
    # without random bits a stochastic format rounds to nearest even (field uploads)
    assert orc.round_storage(v, "bf16sr") == orc.round_storage(v, "bf16") == 1.0


@pytest.mark.parametrize("storage,bracket", [("bf16sr", _bracket_bf16), ("fp16sr", _bracket_f16)])
def test_chain_half_sweep_rounds_each_site_with_its_own_bits(storage, bracket):
    """One half-sweep of an oracle chain: every new value is a bracketing
    grid point of the site's FP64 heat-bath value, and the mean rounding
    error over the sites is zero within its statistical error (the bits used
    are independent of the value)."""
    shape = (16, 12, 10)
    lx, ly, lz = shape
    ch = orc.OracleChain(shape, storage, seed=9, chain=2)
    rng = np.random.default_rng(1)
    ch.set_field(rng.standard_normal((lz, ly, lx)) * 0.5)
    before = ch.phi.copy()
    ch.halfsweep(0)
    lib = orc.load()
    errs, ulps = [], []
    for z in range(lz):
        for y in range(ly):
            for x in range(lx):
                if (x + y + z) & 1:
                    assert ch.phi[z, y, x] == before[z, y, x]
                    continue
                v = lib.orc_site_value(orc._ptr(before), lx, ly, lz, x, y, z, 9, 2, 0)
                lo, hi = bracket(v)
                got = ch.phi[z, y, x]
                assert abs(got) in (lo, hi) and np.sign(got) in (np.sign(v), 0.0), (x, y, z, v, got)
                errs.append(got - v)
                ulps.append(hi - lo)
    errs, ulps = np.array(errs), np.array(ulps)
    r = errs / ulps
    assert abs(r.mean()) <= 4 * r.std() / np.sqrt(r.size)
    assert r.std() > 0.05  # values do round both ways


@pytest.mark.parametrize("storage,spacing_at_1", [("bf16sr", 2.0 ** -7), ("fp16sr", 2.0 ** -10)])
def test_exact_ties_go_by_the_parity_of_the_random_byte(storage, spacing_at_1):
    """A value whose distance past the lower grid point is (k + 1/2)/256 of a
    spacing meets the rule's threshold exactly at u8 = 255 - k: it rounds up
    there when u8 is even and down when it is odd, so over the 256 bytes it
    goes up k + 1 or k times (mean exact on average over k), and the other
    bytes decide as for any value."""
    for k in (0, 1, 76, 77, 200, 255):
        v = 1.0 + (k + 0.5) / 256.0 * spacing_at_1
        u_tie = 255 - k
        ups = np.array([orc.round_storage(v, storage, u) > 1.0 for u in U8])
        assert ups[u_tie] == (u_tie % 2 == 0), (k, u_tie)
        assert np.all(ups[u_tie + 1:]) and not np.any(ups[:u_tie]), k
        assert ups.sum() == (k + 1 if u_tie % 2 == 0 else k)
        assert orc.round_storage(-v, storage, u_tie) == -orc.round_storage(v, storage, u_tie)


@pytest.mark.parametrize("storage", ["bf16sr", "fp16sr"])
def test_no_shrink_or_growth_on_fp32_values(storage):
    """The device rounds FP32 values, which have only 16 (BF16) or 13 (FP16)
    bits below the 16-bit grid, so the rule's threshold is met exactly for
    1/256 or 1/32 of them.  Over a million FP32 values of N(0, 1/4), the
    mean rounding error (exact over the 256 bytes) regressed on the value
    has no slope: below 1.5e-8, where sending every tie up gives +4.4e-8
    (values pushed away from zero, a negative mass term of the same order
    as round-to-nearest-even's shrink for FP16)."""
    rng = np.random.default_rng(4)
    v = (rng.standard_normal(1_000_000) * 0.5).astype(np.float32).astype(np.float64)
    e = orc.round_storage_sr_mean(v, storage) - v
    slope = float(e @ v) / float(v @ v)
    assert abs(slope) < 1.5e-8, slope
