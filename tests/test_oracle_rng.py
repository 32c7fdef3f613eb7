"""Pins of the oracle's random-number path: Philox4x32-10, the uniform grid,
the inverse normal CDF and storage rounding (CPU only)."""

import json
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.special

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")) as f:
        return json.load(f)["vectors"]


@pytest.mark.parametrize("vec", _kat())
def test_philox_known_answers(orc, vec):
    ctr = [int(v, 16) for v in vec["counter"]]
    key = [int(v, 16) for v in vec["key"]]
    out = [int(v, 16) for v in vec["out"]]
    assert list(orc.philox4x32_10(ctr, key)) == out


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "probe")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_probe):
    """An independent Philox4x32-10 (rocRAND's, run on the host) agrees on
    random keys and counters (counter word 1 kept below 2^30, the probe's
    offset range)."""
    rng = np.random.default_rng(7)
    rows = []
    for _ in range(200):
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] %= 2**30
        rows.append((k, c))
    inp = "".join("%x %x %x %x %x %x\n" % (k[0], k[1], c[0], c[1], c[2], c[3]) for k, c in rows)
    res = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True)
    got = [[int(w, 16) for w in line.split()] for line in res.stdout.strip().splitlines()]
    for (k, c), g in zip(rows, got):
        assert list(orc.philox4x32_10(c, k)) == g


def test_site_uniform_counter_layout(orc, rocrand_probe):
    """The site -> (counter, word) assignment: site i = x + lx(y + ly z),
    j = i >> 1, counter (j >> 2, h, chain, 0), word j & 3, r = (k + 1/2) 2^-24
    with k = word >> 8; checked against rocRAND's generator."""
    shape = (10, 6, 5)
    lx, ly, lz = shape
    seed = 0x0123456789ABCDEF
    rng = np.random.default_rng(3)
    cases = []
    for _ in range(100):
        x, y, z = (int(rng.integers(0, n)) for n in shape)
        h = int(rng.integers(0, 1 << 20))
        chain = int(rng.integers(0, 1000))
        cases.append((x, y, z, h, chain))
    inp = ""
    for x, y, z, h, chain in cases:
        j = (x + lx * (y + ly * z)) >> 1
        inp += "%x %x %x %x %x %x\n" % (seed & 0xFFFFFFFF, seed >> 32, j >> 2, h, chain, 0)
    res = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True)
    words = [[int(w, 16) for w in line.split()] for line in res.stdout.strip().splitlines()]
    for (x, y, z, h, chain), w in zip(cases, words):
        j = (x + lx * (y + ly * z)) >> 1
        k = w[j & 3] >> 8
        r_ref = (k + 0.5) * 2.0**-24
        assert orc.site_uniform(shape, x, y, z, seed, chain, h) == r_ref


def test_inverse_cdf_matches_scipy_on_grid(orc):
    """Phi^{-1} on the 24-bit midpoint grid r = (k + 1/2) 2^-24: a dense
    sample including both ends, against scipy.special.ndtri."""
    ks = np.unique(np.concatenate([
        np.arange(0, 4096), np.arange(2**24 - 4096, 2**24),
        np.arange(2**23 - 2048, 2**23 + 2048),
        np.random.default_rng(0).integers(0, 2**24, size=20000)]))
    r = (ks + 0.5) * 2.0**-24
    got = np.array([orc.inv_norm_cdf(v) for v in r])
    ref = scipy.special.ndtri(r)
    err = np.abs(got - ref)
    assert np.all(err <= 4e-15 * np.maximum(np.abs(ref), 1e-3)), err.max()
    # odd symmetry of the grid: r(k) + r(2^24 - 1 - k) = 1
    sym = np.array([orc.inv_norm_cdf((2**24 - 1 - k + 0.5) * 2.0**-24) for k in ks[:500]])
    np.testing.assert_array_equal(sym, -got[:500])


def test_noise_grid_matches_scipy_everywhere(orc):
    """The heat-bath noise Phi^{-1}(r)/sqrt(6) at every one of the 2^24 grid
    points (the reference the device transform is checked against), against
    scipy's ndtri over sqrt(6); odd about the grid's centre."""
    z = orc.noise_grid(0, 1 << 24)
    r = (np.arange(1 << 24) + 0.5) * 2.0**-24
    ref = scipy.special.ndtri(r) / np.sqrt(6.0)
    assert np.max(np.abs(z - ref) / np.abs(ref)) <= 4e-15
    np.testing.assert_array_equal(z[::-1], -z)
    part = orc.noise_grid(12345, 100)
    np.testing.assert_array_equal(part, z[12345:12445])


def test_grid_extremes(orc):
    """Largest |z| on the grid is Phi^{-1}(2^-25) = -5.41998..., and the
    grid has no r = 0 or 1 (no infinities)."""
    z = orc.inv_norm_cdf(2.0**-25)
    assert abs(z - scipy.special.ndtri(2.0**-25)) < 1e-13
    assert -5.42 < z < -5.4199


def test_storage_rounding_fp16_matches_numpy(orc):
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(20000) * 2.0, rng.standard_normal(2000) * 1e-5,
                        rng.standard_normal(2000) * 1e-7, [0.0, -0.0, 6.1e-5, 5.96e-8]])
    got = np.array([orc.round_storage(a, "fp16") for a in v])
    ref = v.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(got, ref)


def test_storage_rounding_fp32(orc):
    rng = np.random.default_rng(6)
    v = rng.standard_normal(5000)
    got = np.array([orc.round_storage(a, "fp32") for a in v])
    np.testing.assert_array_equal(got, v.astype(np.float32).astype(np.float64))


def test_storage_rounding_bf16_halfway_and_torch(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(8)
    # FP32-exact inputs: torch's FP32 -> BF16 conversion is round-to-nearest-even
    v = rng.standard_normal(20000).astype(np.float32).astype(np.float64)
    got = np.array([orc.round_storage(a, "bf16") for a in v])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, ref)
    # exact halfway cases go to the even significand
    one = 1.0
    ulp = 2.0**-7
    assert orc.round_storage(one + ulp / 2, "bf16") == one
    assert orc.round_storage(one + 3 * ulp / 2, "bf16") == one + 2 * ulp
