"""The sample gather fused into the streaming sweep kernel: the loader wave
of each workgroup sums X = sum Q phi and Y = sum S phi^2 over the charged
sites of its tile whose values are final in its plane ring (the colour-0
sites in the colour-1 half-sweep of a measured sweep, the colour-1 sites in
the colour-0 half-sweep of the next sweep; a run's last sample takes its
colour-1 sites from a tail kernel with the same per-tile walk).  Checked
against the separate gather kernel on the same chain (bit-identical fields,
samples equal up to the order of the FP64 sums), the oracle's gather of the
read-back field, graph replays (bit-identical to launch-by-launch runs),
tiling changes between runs, 16-bit storage, measure_every > 1, the
full-size box, and the cases that keep the separate gather."""

import numpy as np
import pytest

import oracle

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
    """Random sites of both colours, every box corner, the first and last
    site of each edge row, and co-located duplicates; charges N(0, 1)."""
    lx, ly, lz = shape
    rng = np.random.default_rng(seed)
    xyz = np.stack([rng.integers(0, lx, n), rng.integers(0, ly, n), rng.integers(0, lz, n)], axis=1)
    corners = np.array([(a, b, c) for a in (0, lx - 1) for b in (0, ly - 1) for c in (0, lz - 1)])
    rows = np.array([(a, ly // 2, lz // 2) for a in (0, 1, lx - 2, lx - 1)])
    xyz = np.concatenate([xyz, corners, rows, xyz[:7]])
    q = rng.standard_normal(len(xyz))
    return xyz.astype(np.int32), q


def _scale(q, phi):
    return float(np.sum(np.abs(q)) ** 2 * max(1.0, np.abs(phi).max()) ** 2)


def _pair(lat_mod, shape, storage, slab, tile, xcd, xyz, q, seed=3, chain=5):
    a = lat_mod.Lattice(shape, storage, seed=seed, chain_id=chain)
    a.set_variant("stream")
    a.set_tuning(slab, tile, xcd)
    b = lat_mod.Lattice(shape, storage, seed=seed, chain_id=chain)
    b.set_variant("zslab")
    for lat in (a, b):
        lat.set_charges(xyz, q)
    return a, b


# FP32 tiles whose plane ring leaves LDS for a (short) staged list without
# losing a resident workgroup per CU; the others keep the separate gather
FP32_FUSING_TILES = (2, 5, 6, 7, 8, 9)

CASES = [
    ((64, 24, 20), "fp32", 0, 9, True),
    ((64, 24, 20), "fp32", 7, 2, False),
    ((64, 24, 20), "fp16", 0, 0, True),
    ((64, 24, 20), "bf16", 5, 4, False),
    ((200, 37, 33), "fp32", 16, 9, True),     # 50 quads per row: a partial 96-quad tile, ragged rows and slab
    ((264, 17, 19), "fp32", 7, 6, True),
    ((136, 13, 7), "fp16", 7, 8, False),     # one slab, 17 quads per row of a 128-quad tile
    ((72, 9, 40), "bf16", 16, 2, True),      # 16-row tiles over 9 rows
    ((520, 12, 5), "fp32", 0, 5, True),      # short lists: a 64-entry LDS stage keeps 3 workgroups per CU
    ((8, 1, 3), "fp32", 0, 2, True),         # one row per plane, one quad per row
    ((64, 24, 20), "fp32", 1, 9, 2),         # one plane per workgroup: the list is read after the last step
    ((64, 24, 20), "fp16", 2, 0, 0),         # two planes: the list is waited for in the last step
    ((200, 37, 33), "bf16", 3, 6, 2),
]


@pytest.mark.parametrize("shape,storage,slab,tile,xcd", CASES)  # xcd: workgroup order (bool = 0 / 1)
def test_fused_gather_matches_separate_and_oracle(lat_mod, shape, storage, slab, tile, xcd):
    print(f"[gpu] fused gather {shape} {storage} slab={slab} tile={tile} xcd={xcd}", flush=True)
    xyz, q = _charges(shape, 60 if tile == 5 else 300, 11)
    a, b = _pair(lat_mod, shape, storage, slab, tile, xcd, xyz, q)
    for lat in (a, b):
        lat.thermalise(5)
        lat.sweep_and_measure(40, 1, 1)
    fused = storage != "fp32" or tile in FP32_FUSING_TILES
    assert a.sample_path() == ("fused" if fused else "separate") and b.sample_path() == "separate"
    fa, fb = a.get_field(), b.get_field()
    np.testing.assert_array_equal(fa, fb)
    sa, sb = a.get_state(), b.get_state()
    assert sa[:2] == sb[:2] == (45, 40)
    tol = 1e-12 * _scale(q, fa)
    assert np.abs(sa[2] - sb[2]).max() <= tol
    # the last sample against the oracle's gather of the read-back field
    ref = oracle.OracleChain(shape)
    ref.phi = fa.astype(np.float64)
    ref.set_charges(xyz, q)
    X, Y = ref.gather()
    Xa, Ya = a.last_measure()
    assert abs(Xa - X) <= 1e-12 * max(1.0, np.sum(np.abs(q)) * np.abs(fa).max())
    assert abs(Ya - Y) <= tol


def test_fused_gather_graphs_and_retiling(lat_mod):
    """Graph replays of fused sweeps are bit-identical to launch-by-launch
    runs; changing the tile or slab between runs rebuilds the per-tile lists
    and the samples stay those of the separate gather."""
    print("[gpu] fused gather graphs + retiling", flush=True)
    shape = (64, 24, 20)
    xyz, q = _charges(shape, 150, 4)
    lats = []
    for mode in (0, 2):
        lat = lat_mod.Lattice(shape, seed=21, chain_id=2)
        lat.set_variant("stream")
        lat.use_graphs(mode)
        lat.set_charges(xyz, q)
        lats.append(lat)
    sep = lat_mod.Lattice(shape, seed=21, chain_id=2)
    sep.set_variant("zslab")
    sep.set_charges(xyz, q)
    tunings = [(0, 9, True), (7, 5, False), (3, 0, True), (20, 2, True), (5, 8, False)]
    for step, (slab, tile, xcd) in enumerate(tunings):
        for lat in lats:
            lat.set_tuning(slab, tile, xcd)
            lat.thermalise(70)
            lat.sweep_and_measure(96, 3, 8)
            assert lat.sample_path() == ("fused" if tile in FP32_FUSING_TILES else "separate")
        sep.thermalise(70)
        sep.sweep_and_measure(96, 3, 8)
        s0, s1, s2 = lats[0].get_state(), lats[1].get_state(), sep.get_state()
        assert s0[0] == s1[0] == s2[0] == 166 * (step + 1)
        np.testing.assert_array_equal(s0[2], s1[2])
        np.testing.assert_array_equal(lats[0].get_field(), lats[1].get_field())
        np.testing.assert_array_equal(lats[0].get_field(), sep.get_field())
        assert np.abs(s0[2] - s2[2]).max() <= 1e-12 * _scale(q, sep.get_field()) * 8
        assert lats[0].last_measure() == lats[1].last_measure()
    # samples every 5th sweep with 2 unmeasured sweeps at the end (the next
    # sweep, not the tail kernel, completes the last sample), then every sweep
    for n, every in ((37, 5), (3, 1), (64, 1)):
        for lat in lats + [sep]:
            lat.sweep_and_measure(n, every, 8)
        s0, s1, s2 = lats[0].get_state(), lats[1].get_state(), sep.get_state()
        assert s0[1] == s1[1] == s2[1]
        np.testing.assert_array_equal(s0[2], s1[2])
        assert np.abs(s0[2] - s2[2]).max() <= 1e-12 * _scale(q, sep.get_field()) * 8
        assert lats[0].last_measure() == lats[1].last_measure()
        X2, Y2 = sep.last_measure()
        assert abs(lats[0].last_measure()[1] - Y2) <= 1e-12 * max(1.0, abs(Y2))


def test_fused_gather_new_charges_and_fallbacks(lat_mod):
    """New charges rebuild the lists; several charge sets, off-lattice
    charges and the other kernels keep the separate gather; an empty charge
    list gives zero samples."""
    print("[gpu] fused gather fallbacks", flush=True)
    shape = (64, 24, 20)
    x1, q1 = _charges(shape, 50, 1)
    x2, q2 = _charges(shape, 80, 2)
    a, b = _pair(lat_mod, shape, "fp32", 0, 9, True, x1, q1)
    for xyz, q in ((x1, q1), (x2, q2)):
        for lat in (a, b):
            lat.set_charges(xyz, q)
            lat.sweep_and_measure(12, 2, 2)
        assert a.sample_path() == "fused"
        sa, sb = a.get_state(), b.get_state()
        assert np.abs(sa[2] - sb[2]).max() <= 2e-12 * _scale(q, a.get_field())
    a.set_charge_sets([(x1, q1), (x2, q2)])
    a.sweep_and_measure(4, 1, 1)
    assert a.sample_path() == "separate"
    a.set_offlattice_charges(x1.astype(np.float64) * 0.5, q1)
    a.sweep_and_measure(4, 1, 1)
    assert a.sample_path() == "separate"
    a.set_charges(x1, q1)
    a.set_variant("quad")
    a.sweep_and_measure(4, 1, 1)
    assert a.sample_path() == "separate"
    a.set_variant("stream")
    a.sweep_and_measure(4, 1, 1)
    assert a.sample_path() == "fused"
    e = lat_mod.Lattice(shape, seed=1)
    e.set_variant("stream")
    e.set_tuning(0, 0, True)  # a tile that fuses only an empty list at FP32
    e.set_charges(np.zeros((0, 3), np.int32), np.zeros(0))
    e.sweep_and_measure(6, 1, 2)
    assert e.sample_path() == "fused"
    _, n, bins = e.get_state()
    assert n == 6 and np.all(bins == 0.0)
    e.set_charges(x1, q1)
    e.sweep_and_measure(2, 1, 2)
    assert e.sample_path() == "separate"


def test_fused_gather_full_size(lat_mod):
    """768^3 on the streaming kernel in its default tiling with the
    benchmark's charge workload: fused samples against the separate gather
    on the same chain."""
    print("[gpu] fused gather 768^3", flush=True)
    from paper_1403_0711_amd import workloads

    c = workloads.largest_subdomain()
    shape, xyz, q = c.shape, c.xyz, c.q
    a = lat_mod.Lattice(shape, seed=77)
    a.set_variant("stream")
    a.set_charges(xyz, q)
    assert a.tuning()["variant"] == "stream"
    a.thermalise(2)
    a.sweep_and_measure(3, 1, 1)
    assert a.sample_path() == "fused"
    sa = a.get_state()
    Xa, Ya = a.last_measure()
    # the oracle's gather of the read-back field (values at the charges'
    # sites passed as a one-row lattice): recursive FP64 sums of n terms
    # differ from any other order by at most (n - 1) 2^-53 sum |terms|, and
    # the per-term products (q phi, (q phi)^2 against S phi^2) by a few ulps
    phi = a.get_field()
    a.close()
    v = np.ascontiguousarray(phi[xyz[:, 2], xyz[:, 1], xyz[:, 0]], dtype=np.float64)
    del phi
    n = v.shape[0]
    line = oracle.OracleChain((n, 1, 1), seed=0)
    line.phi = v.reshape(1, 1, n)
    line.set_charges(np.stack([np.arange(n), np.zeros(n), np.zeros(n)], axis=1), q)
    Xo, Yo = line.gather()
    tol = (n + 4) * 2.0 ** -53
    assert abs(Xa - Xo) <= tol * np.sum(np.abs(q * v)), (Xa, Xo)
    assert abs(Ya - Yo) <= tol * Yo, (Ya, Yo)
    b = lat_mod.Lattice(shape, seed=77)
    b.set_variant("zslab")
    b.set_charges(xyz, q)
    b.thermalise(2)
    b.sweep_and_measure(3, 1, 1)
    sb = b.get_state()
    Xb, Yb = b.last_measure()
    b.close()
    # X sums ~1e6 terms of |q phi| <~ 10: FP64 order differences stay far below 1e-9
    qa = float(np.sum(np.abs(q)))
    assert abs(Xa - Xb) <= 1e-12 * qa * 10.0
    assert abs(Ya - Yb) <= 1e-12 * max(abs(Yb), 1.0)
    assert np.abs(sa[2] - sb[2]).max() <= 1e-12 * (qa * 10.0) ** 2


def test_workgroup_orders_agree(lat_mod):
    """The three workgroup orders over the XCDs (as dealt, a run of tiles per
    XCD, a band of each slab's tiles per XCD) give bit-identical fields and
    samples: partials are kept per tile and summed in a fixed order."""
    print("[gpu] workgroup orders", flush=True)
    for shape, tile, slab in (((64, 40, 20), 9, 5), ((200, 37, 33), 9, 7), ((136, 200, 9), 2, 4)):
        xyz, q = _charges(shape, 200, 6)
        out = []
        for order in (0, 1, 2):
            lat = lat_mod.Lattice(shape, seed=8, chain_id=1)
            lat.set_variant("stream")
            lat.set_tuning(slab, tile, order)
            assert lat.tuning()["xcd_order"] == order
            lat.set_charges(xyz, q)
            lat.thermalise(3)
            lat.sweep_and_measure(10, 1, 2)
            out.append((lat.get_field(), lat.get_state()[2], lat.sample_path()))
        for f, bins, path in out[1:]:
            np.testing.assert_array_equal(f, out[0][0])
            np.testing.assert_array_equal(bins, out[0][1])
            assert path == out[0][2] == "fused"


# Blocked sweep (both half-sweeps per pass): its producer wave gathers a
# sample's colour-0 sites from the colour-0 ring in the sample's own launch
# and its colour-1 sites from the old-plane ring of the next launch; the
# launch after records it.  (shape, storage, planes, rows per tile, order)
BLOCKED_CASES = [
    ((64, 24, 20), "fp32", 0, -1, 2),
    ((64, 24, 20), "fp32", 5, 3, 1),
    ((200, 37, 33), "fp32", 7, 5, 2),   # 25 quads per row, ragged rows and slabs
    ((64, 24, 20), "fp16", 4, 6, 0),
    ((64, 24, 20), "bf16", 3, 2, 2),
    ((8, 1, 3), "fp32", 1, 1, 0),       # one plane per workgroup, one quad per row
    ((96, 37, 23), "fp32", 2, 7, 1),
]


def _blocked_pair(lat_mod, shape, storage, planes, rows, xcd, xyz, q, seed=3, chain=5):
    a = lat_mod.Lattice(shape, storage, seed=seed, chain_id=chain)
    a.set_variant("blocked")
    a.set_tuning(planes, rows, xcd)
    b = lat_mod.Lattice(shape, storage, seed=seed, chain_id=chain)
    b.set_variant("zslab")
    for lat in (a, b):
        lat.set_charges(xyz, q)
    return a, b


@pytest.mark.parametrize("shape,storage,planes,rows,xcd", BLOCKED_CASES)
def test_blocked_fused_gather_matches_separate_and_oracle(lat_mod, shape, storage, planes, rows, xcd):
    print(f"[gpu] blocked fused gather {shape} {storage} planes={planes} rows={rows} xcd={xcd}", flush=True)
    xyz, q = _charges(shape, 300, 12)
    a, b = _blocked_pair(lat_mod, shape, storage, planes, rows, xcd, xyz, q)
    for lat in (a, b):
        lat.thermalise(5)
        lat.sweep_and_measure(40, 1, 1)
    assert a.sample_path() == "fused" and b.sample_path() == "separate"
    fa, fb = a.get_field(), b.get_field()
    np.testing.assert_array_equal(fa, fb)
    sa, sb = a.get_state(), b.get_state()
    assert sa[:2] == sb[:2] == (45, 40)
    tol = 1e-12 * _scale(q, fa)
    assert np.abs(sa[2] - sb[2]).max() <= tol
    ref = oracle.OracleChain(shape)
    ref.phi = fa.astype(np.float64)
    ref.set_charges(xyz, q)
    X, Y = ref.gather()
    Xa, Ya = a.last_measure()
    assert abs(Xa - X) <= 1e-12 * max(1.0, np.sum(np.abs(q)) * np.abs(fa).max())
    assert abs(Ya - Y) <= tol


@pytest.mark.parametrize("shape,planes,rows,n_charges,part_cap", [
    ((64, 24, 20), 7, 5, 3000, 64),    # two or more parts per list
    ((64, 24, 20), 16, 4, 6000, 128),  # four or more parts, ragged last slab
    ((200, 37, 33), 11, 6, 4000, 64),   # ragged rows and slabs
])
def test_blocked_fused_gather_in_parts(lat_mod, monkeypatch, shape, planes, rows, n_charges, part_cap):
    """Charge lists staged in several parts (a part restaged in the step
    before its first one): samples equal to the separate gather's and the
    oracle's, fields bit-identical."""
    print(f"[gpu] blocked fused gather in parts {shape} planes={planes} rows={rows} "
          f"charges={n_charges} cap={part_cap}", flush=True)
    monkeypatch.setenv("LATCOUL_GATHER_PART_CAP", str(part_cap))
    xyz, q = _charges(shape, n_charges, 31)
    a, b = _blocked_pair(lat_mod, shape, "fp32", planes, rows, 1, xyz, q)
    parts, entries = a.gather_parts()
    assert parts >= 2 and 0 < entries <= max(64, part_cap)
    for lat in (a, b):
        lat.thermalise(3)
        lat.sweep_and_measure(25, 1, 1)
    assert a.sample_path() == "fused" and b.sample_path() == "separate"
    fa = a.get_field()
    np.testing.assert_array_equal(fa, b.get_field())
    sa, sb = a.get_state(), b.get_state()
    assert np.abs(sa[2] - sb[2]).max() <= 1e-12 * _scale(q, fa)
    ref = oracle.OracleChain(shape)
    ref.phi = fa.astype(np.float64)
    ref.set_charges(xyz, q)
    X, Y = ref.gather()
    Xa, Ya = a.last_measure()
    assert abs(Xa - X) <= 1e-12 * max(1.0, np.sum(np.abs(q)) * np.abs(fa).max())
    assert abs(Ya - Y) <= 1e-12 * _scale(q, fa)


def test_blocked_fused_gather_graphs_and_retiling(lat_mod):
    """Blocked sweeps with the fused gather: graph replays bit-identical to
    launch-by-launch runs, tiling changes between runs, samples every k-th
    sweep (a sample whose colour-1 sites the next launch gathers, recorded by
    the one after or by the call's tail), all equal to the separate gather."""
    print("[gpu] blocked fused gather graphs + retiling", flush=True)
    shape = (64, 24, 20)
    xyz, q = _charges(shape, 150, 5)
    lats = []
    for mode in (0, 2):
        lat = lat_mod.Lattice(shape, seed=21, chain_id=2)
        lat.set_variant("blocked")
        lat.use_graphs(mode)
        lat.set_charges(xyz, q)
        lats.append(lat)
    sep = lat_mod.Lattice(shape, seed=21, chain_id=2)
    sep.set_variant("zslab")
    sep.set_charges(xyz, q)
    for step, (planes, rows, xcd) in enumerate([(0, -1, 2), (7, 5, 1), (3, 2, 0), (20, 16, 2)]):
        for lat in lats:
            lat.set_tuning(planes, rows, xcd)
            lat.thermalise(70)
            lat.sweep_and_measure(96, 3, 8)
            assert lat.sample_path() == "fused"
        sep.thermalise(70)
        sep.sweep_and_measure(96, 3, 8)
        s0, s1, s2 = lats[0].get_state(), lats[1].get_state(), sep.get_state()
        assert s0[0] == s1[0] == s2[0] == 166 * (step + 1)
        np.testing.assert_array_equal(s0[2], s1[2])
        np.testing.assert_array_equal(lats[0].get_field(), lats[1].get_field())
        np.testing.assert_array_equal(lats[0].get_field(), sep.get_field())
        assert np.abs(s0[2] - s2[2]).max() <= 1e-12 * _scale(q, sep.get_field()) * 8
        assert lats[0].last_measure() == lats[1].last_measure()
    for n, every in ((37, 5), (3, 1), (1, 1), (2, 2), (64, 1), (10, 4)):
        for lat in lats + [sep]:
            lat.sweep_and_measure(n, every, 8)
        s0, s1, s2 = lats[0].get_state(), lats[1].get_state(), sep.get_state()
        assert s0[1] == s1[1] == s2[1]
        np.testing.assert_array_equal(s0[2], s1[2])
        assert np.abs(s0[2] - s2[2]).max() <= 1e-12 * _scale(q, sep.get_field()) * 8
        assert lats[0].last_measure() == lats[1].last_measure()
        X2, Y2 = sep.last_measure()
        assert abs(lats[0].last_measure()[1] - Y2) <= 1e-12 * max(1.0, abs(Y2))


def test_blocked_fused_gather_full_size(lat_mod):
    """768^3 with the benchmark's charges on the blocked sweep in its default
    configuration: fused samples against the oracle's gather of the
    read-back field, and against the separate gather of the streaming
    kernel on the same chain."""
    print("[gpu] blocked fused gather 768^3", flush=True)
    from paper_1403_0711_amd import workloads

    c = workloads.largest_subdomain()
    shape, xyz, q = c.shape, c.xyz, c.q
    a = lat_mod.Lattice(shape, seed=77)
    a.set_variant("blocked")
    a.set_charges(xyz, q)
    a.thermalise(2)
    a.sweep_and_measure(3, 1, 1)
    assert a.sample_path() == "fused"
    print("[gpu] staged parts, entries per part:", a.gather_parts(), flush=True)
    assert a.gather_parts()[0] >= 1
    sa = a.get_state()
    Xa, Ya = a.last_measure()
    phi = a.get_field()
    a.close()
    v = np.ascontiguousarray(phi[xyz[:, 2], xyz[:, 1], xyz[:, 0]], dtype=np.float64)
    del phi
    n = v.shape[0]
    line = oracle.OracleChain((n, 1, 1), seed=0)
    line.phi = v.reshape(1, 1, n)
    line.set_charges(np.stack([np.arange(n), np.zeros(n), np.zeros(n)], axis=1), q)
    Xo, Yo = line.gather()
    tol = (n + 4) * 2.0 ** -53
    assert abs(Xa - Xo) <= tol * np.sum(np.abs(q * v)), (Xa, Xo)
    assert abs(Ya - Yo) <= tol * Yo, (Ya, Yo)
    b = lat_mod.Lattice(shape, seed=77)
    b.set_variant("stream")
    b.set_charges(xyz, q)
    b.thermalise(2)
    b.sweep_and_measure(3, 1, 1)
    sb = b.get_state()
    b.close()
    qa = float(np.sum(np.abs(q)))
    assert np.abs(sa[2] - sb[2]).max() <= 1e-12 * (qa * 10.0) ** 2


def _sets_of(shape, seed):
    """Four charge sets: random sites with co-located duplicates, a second
    random set, an empty set, and one that shares sites with the first."""
    xyz, q = _charges(shape, 200, seed)
    xyz2, q2 = _charges(shape, 120, seed + 1)
    rng = np.random.default_rng(seed + 2)
    xyz4 = np.concatenate([xyz[:50], xyz2[:10]])
    q4 = rng.standard_normal(len(xyz4))
    return [(xyz, q), (xyz2, q2), (np.zeros((0, 3), np.int32), np.zeros(0)), (xyz4, q4)]


@pytest.mark.parametrize("shape,storage,planes,rows,xcd", [
    ((64, 24, 20), "fp32", 0, -1, 2),
    ((200, 37, 33), "fp32", 7, 5, 2),   # ragged rows and slabs
    ((64, 24, 20), "fp16sr", 4, 6, 0),
    ((96, 37, 23), "bf16", 2, 7, 1),
])
def test_blocked_fused_gather_charge_sets(lat_mod, shape, storage, planes, rows, xcd):
    """Several charge sets (up to four) gathered in the blocked sweep's one
    walk, each entry tagged with its set: fields bit-identical to the
    separate gather's chain, every set's samples equal to its samples there
    (FP64 sums in another order), the empty set's samples zero, across a
    graph chunk and the eager sweeps after it."""
    print(f"[gpu] blocked fused gather, charge sets {shape} {storage} planes={planes} rows={rows}", flush=True)
    sets = _sets_of(shape, 21)
    a = lat_mod.Lattice(shape, storage, seed=3, chain_id=5)
    a.set_variant("blocked")
    a.set_tuning(planes, rows, xcd)
    b = lat_mod.Lattice(shape, storage, seed=3, chain_id=5)
    b.set_variant("zslab")
    for lat in (a, b):
        lat.set_charge_sets(sets)
        lat.thermalise(5)
        lat.sweep_and_measure(40, 1, 1)
    assert a.sample_path() == "fused" and b.sample_path() == "separate"
    fa = a.get_field()
    np.testing.assert_array_equal(fa, b.get_field())
    sa, sb = a.get_state(), b.get_state()
    assert sa[:2] == sb[:2] == (45, 40) and sa[2].shape == (4, 40, 2)
    for k, (xyz, q) in enumerate(sets):
        tol = 1e-12 * max(1.0, _scale(q, fa))
        assert np.abs(sa[2][k] - sb[2][k]).max() <= tol, k
        ma, mb = a.energy_estimate(charge_set=k)[0], b.energy_estimate(charge_set=k)[0]
        assert abs(ma - mb) <= tol, k
    assert np.all(sa[2][2] == 0.0)
    # the last sample of set 0 against the oracle's gather of the read-back field
    ref = oracle.OracleChain(shape)
    ref.phi = fa.astype(np.float64)
    ref.set_charges(*sets[0])
    X, Y = ref.gather()
    O = sa[2][0][-1]
    assert abs((O[0] - O[1]) - (X * X - Y)) <= 1e-10 * _scale(sets[0][1], fa)


def test_blocked_fused_gather_charge_sets_in_parts_and_limits(lat_mod, monkeypatch):
    """Four sets whose lists are staged in several parts give the separate
    gather's samples; five sets (more than the walk serves) keep the
    separate gather."""
    print("[gpu] blocked fused gather, charge sets in parts; five sets", flush=True)
    shape = (64, 24, 20)
    monkeypatch.setenv("LATCOUL_GATHER_PART_CAP", "64")
    sets = [_charges(shape, 1200, s) for s in (5, 6, 7)] + [(np.zeros((0, 3), np.int32), np.zeros(0))]
    a = lat_mod.Lattice(shape, seed=8, chain_id=1)
    a.set_variant("blocked")
    a.set_tuning(11, 4, 1)
    b = lat_mod.Lattice(shape, seed=8, chain_id=1)
    b.set_variant("zslab")
    for lat in (a, b):
        lat.set_charge_sets(sets)
        lat.sweep_and_measure(30, 1, 1)
    assert a.sample_path() == "fused" and a.gather_parts()[0] >= 2
    fa = a.get_field()
    np.testing.assert_array_equal(fa, b.get_field())
    sa, sb = a.get_state()[2], b.get_state()[2]
    for k, (xyz, q) in enumerate(sets):
        assert np.abs(sa[k] - sb[k]).max() <= 1e-12 * max(1.0, _scale(q, fa)), k
    five = lat_mod.Lattice(shape, seed=8, chain_id=1)
    five.set_variant("blocked")
    five.set_charge_sets(sets + [sets[0]])
    five.sweep_and_measure(4, 1, 1)
    assert five.sample_path() == "separate"
