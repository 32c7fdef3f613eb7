"""The allocation-free entry point sweep_and_measure_noalloc against
sweep_and_measure, through the C ABI: same field bit for bit and same
samples (sums up to FP64 summation order) on two calls in a row, the second
on a smaller lattice with another sample path, with no allocator call during
either; its documented refusals."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lat_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_0711_amd import lattice

    lattice.load_library()
    return lattice


def _charges(shape, n, seed):
    from paper_1403_0711_amd import workloads

    rng = np.random.default_rng(seed)
    xyz = workloads.distinct_sites(rng, n, (0, 0, 0), shape)
    q = rng.standard_normal(n)
    return xyz, q - q.mean()


def _pair(lat_mod, shape, variant, sets, seed, tuning=None):
    """Two identical lattices (same seed, charges, warm-up): one for each
    entry point."""
    out = []
    for _ in range(2):
        lat = lat_mod.Lattice(shape, seed=seed, chain_id=5)
        lat.set_variant(variant)
        if tuning:
            lat.set_tuning(*tuning)
        if len(sets) == 1:
            lat.set_charges(*sets[0])
        else:
            lat.set_charge_sets(sets)
        lat.thermalise(3)
        lat.sweep_and_measure(6, 1, 2)  # grows the bins to their first size (64 bins)
        out.append(lat)
    return out


def _compare(a, b):
    np.testing.assert_array_equal(a.get_field(), b.get_field())
    ta, na, ba = a.get_state()
    tb, nb, bb = b.get_state()
    assert (ta, na) == (tb, nb)
    np.testing.assert_allclose(ba, bb, rtol=1e-12, atol=1e-12 * max(1.0, float(np.abs(bb).max())))


def test_noalloc_matches_sweep_and_measure(lat_mod):
    print("[gpu] no-alloc: streaming kernel, fused gather, 128x40x24", flush=True)
    shape = (128, 40, 24)
    # 96-quad tiles, 5 planes per workgroup: a tiling whose lists fuse at FP32
    a, b = _pair(lat_mod, shape, "stream", [_charges(shape, 300, 1)], seed=21, tuning=(5, 9, 1))
    before = a._mem.n_alloc
    a.sweep_and_measure_noalloc(20, 1, 2)
    b.sweep_and_measure(20, 1, 2)
    assert a._mem.n_alloc == before
    assert a.sample_path() == b.sample_path() == "fused"
    _compare(a, b)
    a.close()
    b.close()

    print("[gpu] no-alloc: smaller lattice, quad kernel, three charge sets", flush=True)
    shape = (32, 16, 8)
    sets = [_charges(shape, 40, s) for s in (2, 3, 4)]
    a, b = _pair(lat_mod, shape, "quad", sets, seed=22)
    before = a._mem.n_alloc
    a.sweep_and_measure_noalloc(12, 2, 2)
    b.sweep_and_measure(12, 2, 2)
    assert a._mem.n_alloc == before
    assert a.sample_path() == "separate"
    _compare(a, b)
    for k in range(3):
        ma = a.energy_estimate(allow_few_bins=True, charge_set=k)
        mb = b.energy_estimate(allow_few_bins=True, charge_set=k)
        assert ma[2:] == mb[2:]
        assert abs(ma[0] - mb[0]) <= 1e-12 * max(1.0, abs(mb[0]))
    a.close()
    b.close()


def test_noalloc_blocked_charge_sets(lat_mod):
    """Several charge sets gathered inside the blocked sweep (the call's
    last sample through the separate gather): the allocation-free entry
    point gives the same field and samples, on two calls in a row."""
    print("[gpu] no-alloc: blocked sweep, three charge sets gathered in the sweep", flush=True)
    shape = (64, 24, 20)
    sets = [_charges(shape, 200, s) for s in (6, 7, 8)]
    a, b = _pair(lat_mod, shape, "blocked", sets, seed=24, tuning=(7, 4, 1))
    before = a._mem.n_alloc
    for n in (20, 9):
        a.sweep_and_measure_noalloc(n, 1, 2)
        b.sweep_and_measure(n, 1, 2)
        assert a._mem.n_alloc == before
        assert a.sample_path() == b.sample_path() == "fused"
        _compare(a, b)
    a.close()
    b.close()


def test_noalloc_resident_and_refusals(lat_mod):
    print("[gpu] no-alloc: resident kernel and refusals", flush=True)
    shape = (16, 16, 16)
    a, b = _pair(lat_mod, shape, "resident", [_charges(shape, 8, 5)], seed=23)
    a.sweep_and_measure_noalloc(30, 1, 2)
    b.sweep_and_measure(30, 1, 2)
    _compare(a, b)
    with pytest.raises(lat_mod.LatticeError) as e:  # 6 + 30 + 100 samples: more than 64 bins of 2
        a.sweep_and_measure_noalloc(100, 1, 2)
    assert "room" in str(e.value)
    with pytest.raises(lat_mod.LatticeError):
        a.sweep_and_measure_noalloc(2, 1, 3)  # another bin size
    a.close()
    b.close()
    c = lat_mod.Lattice(shape, seed=1)
    with pytest.raises(lat_mod.LatticeError) as e:
        c.sweep_and_measure_noalloc(2, 1, 1)
    assert "charges" in str(e.value)
    c.close()
