"""Off-lattice charges and forces through the C ABI (a charge at an arbitrary
position spread over the 8 corners of its cell; forces from the gradient of
the interpolant): per-sweep samples and force sums against the oracle's chain,
integer positions against on-lattice charges, estimates against the exact
interpolated lattice energy and its gradient, graph replays, errors."""

import math

import numpy as np
import pytest

import oracle
from oracle import exact

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
    rng = np.random.default_rng(seed)
    hi = np.array(shape, dtype=np.float64) - 1.0
    r = rng.uniform(size=(n, 3)) * hi
    r[0] = [0.0, 0.0, 0.0]          # a box corner
    r[1] = hi                       # the far corner (clamped top cell, fraction 1)
    r[2] = np.floor(hi / 2)         # an integer position
    q = rng.standard_normal(n)
    return r, q - q.mean()


@pytest.mark.parametrize("variant", ["auto", "generic", "stream", "blocked"])
def test_offlattice_samples_and_forces_match_oracle(lat_mod, variant):
    print(f"[gpu] off-lattice vs oracle {variant}", flush=True)
    shape = (16, 10, 8) if variant != "generic" else (14, 9, 7)
    r, q = _charges(shape, 12, 1)
    lat = lat_mod.Lattice(shape, seed=31, chain_id=6)
    lat.set_variant(variant)
    lat.set_offlattice_charges(r, q, forces=True)
    ref = oracle.OracleChain(shape, seed=31, chain=6)
    lat.thermalise(4)
    ref.sweeps(4)
    S = 25
    lat.sweep_and_measure(S, 1, 1)
    got = lat.get_state()[2]
    got = got[:, 0] - got[:, 1]
    want, fsum = np.zeros(S), np.zeros((12, 3))
    for s in range(S):
        ref.sweeps(1)
        X, Y, phit, grad = oracle.gather_offlattice(ref.phi, r, q)
        want[s] = X * X - Y
        fsum += oracle.force_sample(X, phit, grad, q)
    scale = np.abs(q).sum() ** 2 * np.abs(ref.phi).max() ** 2
    assert np.abs(got - want).max() <= 1e-4 * scale
    g, se, m = lat.force_estimate()
    assert m == S and g.shape == (12, 3) and np.all(se >= 0)
    assert np.abs(g - fsum / S).max() <= 1e-4 * scale
    X_last, _ = lat.last_measure()
    assert abs(X_last - X) <= 1e-4 * math.sqrt(scale)


def test_integer_positions_equal_site_charges(lat_mod):
    print("[gpu] off-lattice at sites", flush=True)
    shape = (24, 12, 10)
    rng = np.random.default_rng(2)
    xyz = np.stack([rng.integers(0, s, 30) for s in shape], axis=1)
    xyz = np.unique(xyz, axis=0)
    q = rng.standard_normal(xyz.shape[0])
    a = lat_mod.Lattice(shape, seed=4)
    b = lat_mod.Lattice(shape, seed=4)
    for lat in (a, b):
        lat.set_variant("quad")
    a.set_charges(xyz, q)
    b.set_offlattice_charges(xyz.astype(np.float64), q)
    for lat in (a, b):
        lat.sweep_and_measure(40, 1, 1)
    sa, sb = a.get_state()[2], b.get_state()[2]
    oa, ob = sa[:, 0] - sa[:, 1], sb[:, 0] - sb[:, 1]
    assert np.abs(oa - ob).max() <= 1e-12 * max(1.0, np.abs(oa).max())


def test_offlattice_estimates_match_exact(lat_mod):
    """Energy and dE/dr of four off-lattice charges on an 8^3 box against the
    exact interpolated lattice values (Cholesky Green's function)."""
    print("[gpu] off-lattice vs exact", flush=True)
    shape = (8, 8, 8)
    r = np.array([[2.5, 3.25, 4.0], [4.75, 4.1, 3.3], [3.2, 5.6, 2.4], [5.5, 2.2, 5.1]])
    q = np.array([1.0, 1.0, -1.0, -1.0])
    G = exact.green_dense(shape)
    e = exact.energy_offlattice_dense(shape, r, q, G)
    grad = exact.grad_offlattice_dense(shape, r, q, G)
    lat = lat_mod.Lattice(shape, seed=9)
    lat.set_offlattice_charges(r, q, forces=True)
    lat.thermalise(200)
    lat.sweep_and_measure(300000, 3, 1000)
    m, se, M, nb = lat.energy_estimate()
    assert M == 100000 and nb == 100
    assert abs(m - e) <= 4 * se, (m, e, se)
    g, gse, n = lat.force_estimate()
    assert n == 100000
    assert np.all(np.abs(g - grad) <= 6 * gse + 1e-9), (g, grad, gse)


def test_offlattice_graph_replays_and_errors(lat_mod):
    print("[gpu] off-lattice graphs + errors", flush=True)
    shape = (64, 24, 20)
    r, q = _charges(shape, 40, 3)
    lats = []
    for mode in (0, 2):
        lat = lat_mod.Lattice(shape, seed=12)
        lat.set_variant("quad")
        lat.use_graphs(mode)
        lat.set_offlattice_charges(r, q, forces=True)
        lats.append(lat)
    for _ in range(3):
        for lat in lats:
            lat.sweep_and_measure(96, 3, 4)
    np.testing.assert_array_equal(lats[0].get_state()[2], lats[1].get_state()[2])
    g0, g1 = lats[0].force_estimate(), lats[1].force_estimate()
    np.testing.assert_array_equal(g0[0], g1[0])
    assert g0[2] == g1[2] == 96
    lat = lats[0]
    with pytest.raises(lat_mod.LatticeError):
        lat.set_offlattice_charges([[64.0, 0.0, 0.0]], [1.0])  # x > lx - 1
    with pytest.raises(lat_mod.LatticeError):
        lat.set_offlattice_charges([[1.0, -0.5, 0.0]], [1.0])
    with pytest.raises(lat_mod.LatticeError):
        lat.set_offlattice_charges([[1.0, 1.0, 1.0]], [np.nan])
    with pytest.raises(lat_mod.LatticeError):
        lat.set_variant("resident")
    lat.set_offlattice_charges(r, q)  # forces off
    with pytest.raises(lat_mod.LatticeError):
        lat.force_estimate()
    flat = lat_mod.Lattice((8, 1, 4))
    with pytest.raises(lat_mod.LatticeError):
        flat.set_offlattice_charges([[1.0, 0.0, 1.0]], [1.0])  # an edge of 1
    small = lat_mod.Lattice((16, 16, 16))
    small.set_offlattice_charges([[1.5, 2.5, 3.5]], [1.0])
    assert small.tuning()["variant"] != "resident"
    small.set_charges([[1, 2, 3]], [1.0])
    assert small.tuning()["variant"] == "resident"
