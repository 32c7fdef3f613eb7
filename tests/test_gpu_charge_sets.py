"""Several charge sets measured on one field chain (the paper's reuse of the
same field samples for any charge configuration), through the C ABI: each
set's samples equal those of a lattice holding that set alone, and the
oracle's gather of the same chain; graph replays, checkpoints and argument
errors."""

import numpy as np
import pytest

import oracle
from paper_1403_0711_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lat_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_0711_amd import lattice

    lattice.load_library()
    return lattice


def _sets(shape, seed=0):
    """Four sets: neutral +-1, a same-sign blob, an empty set, and a set with
    co-located charges."""
    lx, ly, lz = shape
    a = workloads.small_neutral(seed=seed, L=min(shape), n=12)
    b = workloads.gaussian_blob(seed=seed + 1, L=min(shape), n=40, sigma=min(shape) / 6)
    rng = np.random.default_rng(seed + 2)
    xyz = workloads.distinct_sites(rng, 10, (0, 0, 0), shape)
    d_xyz = np.concatenate([xyz, xyz[:4]])
    d_q = np.concatenate([rng.standard_normal(10), np.linspace(-1, 1, 4)])
    return [(a.xyz, a.q), (b.xyz, b.q), (np.zeros((0, 3), np.int32), np.zeros(0)), (d_xyz, d_q)]


def _series(bins):
    return bins[..., 0] - bins[..., 1]


@pytest.mark.parametrize("variant", ["auto", "stream", "generic", "blocked"])
def test_sets_equal_single_set_lattices(lat_mod, variant):
    print(f"[gpu] charge sets vs single sets {variant}", flush=True)
    shape = (32, 24, 20) if variant != "generic" else (30, 14, 9)
    sets = _sets(shape)
    lat = lat_mod.Lattice(shape, seed=5, chain_id=2)
    lat.set_variant(variant)
    lat.set_charge_sets(sets)
    lat.thermalise(5)
    lat.sweep_and_measure(40, 1, 1)
    _, n, bins = lat.get_state()
    assert n == 40 and bins.shape == (4, 40, 2)
    for k, (xyz, q) in enumerate(sets):
        one = lat_mod.Lattice(shape, seed=5, chain_id=2)
        one.set_variant(variant if variant != "auto" else "quad")
        one.set_charges(xyz, q)
        one.thermalise(5)
        one.sweep_and_measure(40, 1, 1)
        ref = _series(one.get_state()[2])
        got = _series(bins[k])
        scale = max(np.abs(ref).max(), 1.0)
        assert np.abs(got - ref).max() <= 1e-12 * scale, k
        if k == 2:
            assert np.all(got == 0.0)  # empty set: X = Y = 0
        one.close()
        m, se, M, nb = lat.energy_estimate(charge_set=k)
        assert M == 40 and nb == 40
        assert abs(m - got.mean()) <= 1e-12 * scale
    with pytest.raises(lat_mod.LatticeError):
        lat.energy_estimate(charge_set=4)


def test_sets_match_oracle_chain(lat_mod):
    """Per-sweep samples of each set against the oracle's gather of its own
    chain (FP64): equal to the FP32-vs-FP64 field tolerance."""
    print("[gpu] charge sets vs oracle", flush=True)
    shape = (16, 16, 16)
    sets = _sets(shape, seed=3)
    lat = lat_mod.Lattice(shape, seed=77, chain_id=1)
    lat.set_charge_sets(sets)
    assert lat.tuning()["variant"] != "resident"  # one charge set only there
    lat.sweep_and_measure(30, 1, 1)
    got = _series(lat.get_state()[2])
    ref = oracle.OracleChain(shape, seed=77, chain=1)
    want = np.zeros((len(sets), 30))
    for s in range(30):
        ref.sweeps(1)
        for k, (xyz, q) in enumerate(sets):
            ref.set_charges(xyz, q)
            X, Y = ref.gather()
            want[k, s] = X * X - Y
    phi_max = np.abs(ref.phi).max()
    for k, (xyz, q) in enumerate(sets):
        scale = (np.abs(q).sum() ** 2) * phi_max ** 2 + 1e-30
        assert np.abs(got[k] - want[k]).max() <= 1e-4 * scale, k


def test_sets_graph_replays_and_checkpoint(lat_mod):
    """Graph-captured chunks measure every set as launch-by-launch runs do;
    a checkpoint of all sets' bins restores bit-identically."""
    print("[gpu] charge sets graphs + checkpoint", flush=True)
    shape = (64, 24, 20)
    sets = _sets(shape, seed=9)
    lats = []
    for mode in (0, 2):
        lat = lat_mod.Lattice(shape, seed=21)
        lat.set_variant("quad")
        lat.use_graphs(mode)
        lat.set_charge_sets(sets)
        lats.append(lat)
    for _ in range(3):
        for lat in lats:
            lat.sweep_and_measure(96, 3, 4)
    s0, s1 = lats[0].get_state(), lats[1].get_state()
    assert s0[0] == s1[0] and s0[1] == s1[1] == 96
    np.testing.assert_array_equal(s0[2], s1[2])
    # checkpoint: field + state into a fresh lattice, continue both
    field = lats[0].get_field()
    c = lat_mod.Lattice(shape, seed=21)
    c.set_variant("quad")
    c.set_charge_sets(sets)
    c.set_field(field)
    c.set_state(s0[0], s0[1], 4, s0[2])
    for lat in (lats[0], c):
        lat.sweep_and_measure(30, 3, 4)
    np.testing.assert_array_equal(lats[0].get_state()[2], c.get_state()[2])
    for k in range(len(sets)):
        assert lats[0].energy_estimate(charge_set=k) == c.energy_estimate(charge_set=k)


def test_charge_set_errors(lat_mod):
    print("[gpu] charge set errors", flush=True)
    lat = lat_mod.Lattice((16, 16, 16), seed=1)
    with pytest.raises(lat_mod.LatticeError):
        lat.set_charge_sets([])  # no set
    lat.set_variant("resident")
    with pytest.raises(lat_mod.LatticeError):
        lat.set_charge_sets(_sets((16, 16, 16)))
    lat.set_variant("auto")
    lat.set_charge_sets(_sets((16, 16, 16)))
    with pytest.raises(lat_mod.LatticeError):
        lat.set_variant("resident")
    with pytest.raises(lat_mod.LatticeError):
        lat.set_charge_sets([([[16, 0, 0]], [1.0])])  # outside the box
    assert lat.n_sets == 4  # a failed call leaves the sets in place
    lat.set_charges([[1, 1, 1]], [1.0])
    assert lat.n_sets == 1
    lat.set_variant("resident")
