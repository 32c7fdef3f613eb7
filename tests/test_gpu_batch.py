"""GPU parity of the batched-chain path (one persistent launch, one workgroup
per chain) against single lattices and the CPU oracle, through the C ABI."""

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


EDGES = [(24, 24, 24), (16, 8, 12), (10, 6, 5), (32, 32, 32), (2, 1, 1), (40, 16, 9)]


def _charges(shape, n, seed):
    rng = np.random.default_rng(seed)
    xyz = workloads.distinct_sites(rng, n, (0, 0, 0), shape)
    q = rng.standard_normal(n)
    return xyz, q - q.mean()


def test_batch_matches_single_lattices(lat_mod):
    """Each chain of a batch equals a single lattice with the same seed and
    chain id: same field after every run, same estimate."""
    print("[gpu] batch vs single lattices", flush=True)
    seed = 12345
    ids = [7, 0, 3, 1000, 5, 2]
    b = lat_mod.Batch(EDGES, "fp32", seed=seed, chain_ids=ids)
    singles = []
    for k, e in enumerate(EDGES):
        n = min(6, int(np.prod(e)))
        xyz, q = _charges(e, n, k)
        b.set_charges(k, xyz, q)
        s = lat_mod.Lattice(e, "fp32", seed=seed, chain_id=ids[k])
        s.set_charges(xyz, q)
        singles.append(s)
    b.run(5, 20, 5)
    for s in singles:
        s.thermalise(5)
        s.sweep_and_measure(20, 1, 5)
    for k, s in enumerate(singles):
        fb, fs = b.get_field(k), s.get_field()
        assert np.abs(fb - fs).max() <= 1e-6 * max(np.abs(fs).max(), 1e-30), k
        mb, seb, Mb, nbb = b.energy_estimate(k)
        ms, ses, Ms, nbs = s.energy_estimate()
        assert (Mb, nbb) == (Ms, nbs) == (20, 4)
        assert abs(mb - ms) <= 1e-6 * max(1.0, abs(ms)), k
    # a second run continues the same streams
    b.run(0, 10, 5)
    for s in singles:
        s.sweep_and_measure(10, 1, 5)
    for k, s in enumerate(singles):
        assert np.abs(b.get_field(k) - s.get_field()).max() <= 1e-6 * max(np.abs(s.get_field()).max(), 1e-30)
        assert b.energy_estimate(k)[2] == 30


# chains past the single-workgroup size, so that the single lattices run the
# quad kernel: at most 3072 quads per plane (the LDS ring path; 128 x 64 with
# a first window of exactly the two kept chunks, 136 x 64 one past them,
# 192 x 128 at the ring's full span of 3072, 48 x 40 over eight chunks with a
# ragged last one) and wider planes (200 x 128: 3200 quads, the
# two-quads-per-thread path)
RING_EDGES = [(128, 64, 4), (136, 64, 3), (48, 40, 30), (32, 32, 32), (192, 128, 2), (200, 128, 2)]


# 64^3 chains that bring a batch's fields to the 256 MiB at which the batch
# sweeps through the LDS ring (two 64^3 colour arrays: 1 MiB at FP32)
def _fillers(storage):
    return [(64, 64, 64)] * (256 if storage == "fp32" else 512)


@pytest.mark.parametrize("storage,filled", [("fp32", False), ("fp32", True), ("bf16", True), ("fp16", True),
                                            ("bf16sr", True), ("fp16sr", False)])
def test_batch_ring_matches_quad_kernel(lat_mod, storage, filled):
    """Batched chains equal single lattices swept by the quad kernel, bit for
    bit: in a small batch (the half-sweep from memory) and in batches filled
    to the size that takes the LDS ring, in every storage format, on both
    sides of the ring's plane limit."""
    print(f"[gpu] batch vs quad kernel {storage} filled={filled}", flush=True)
    seed = 777
    ids = [3, 11, 0, 42, 7, 8]
    edges = RING_EDGES + (_fillers(storage) if filled else [])
    b = lat_mod.Batch(edges, storage, seed=seed,
                      chain_ids=ids + list(range(100, 100 + len(edges) - len(ids))))
    singles = []
    for k, e in enumerate(RING_EDGES):
        xyz, q = _charges(e, 8, 100 + k)
        b.set_charges(k, xyz, q)
        s = lat_mod.Lattice(e, storage, seed=seed, chain_id=ids[k])
        s.set_variant("quad")
        s.set_charges(xyz, q)
        singles.append(s)
    b.run(3, 6, 3)
    for s in singles:
        s.thermalise(3)
        s.sweep_and_measure(6, 1, 3)
    for k, s in enumerate(singles):
        assert np.array_equal(b.get_field(k), s.get_field()), (storage, RING_EDGES[k])
        mb, Mb = b.energy_estimate(k)[0], b.energy_estimate(k)[2]
        ms, Ms = s.energy_estimate()[0], s.energy_estimate()[2]
        assert Mb == Ms == 6
        assert abs(mb - ms) <= 1e-9 * max(1.0, abs(ms)), (storage, RING_EDGES[k])


def test_batch_autotuned_matches_quad_kernel(lat_mod):
    """A batch whose half-sweep form the autotuner chose per box (the boxes
    on both sides of the ring's plane limit, several chains of some) gives
    the single lattices' fields and samples bit for bit, as the untuned batch
    does; a second autotune of the same batch reuses the cached choices."""
    print("[gpu] autotuned batch vs quad kernel", flush=True)
    seed = 4242
    edges = RING_EDGES + [(64, 64, 64)] * 4 + [(48, 40, 30)] * 3
    ids = list(range(20, 20 + len(edges)))
    tuned = lat_mod.Batch(edges, "fp32", seed=seed, chain_ids=ids)
    plain = lat_mod.Batch(edges, "fp32", seed=seed, chain_ids=ids)
    n_ring = tuned.autotune(2)
    assert 0 <= n_ring <= len(edges)
    assert tuned.autotune(2) == n_ring
    singles = []
    for k, e in enumerate(edges):
        xyz, q = _charges(e, 8, 300 + k)
        tuned.set_charges(k, xyz, q)
        plain.set_charges(k, xyz, q)
        if k < len(RING_EDGES):
            s = lat_mod.Lattice(e, "fp32", seed=seed, chain_id=ids[k])
            s.set_variant("quad")
            s.set_charges(xyz, q)
            singles.append(s)
    for b in (tuned, plain):
        b.run(2, 6, 3)
    for s in singles:
        s.thermalise(2)
        s.sweep_and_measure(6, 1, 3)
    for k in range(len(edges)):
        assert np.array_equal(tuned.get_field(k), plain.get_field(k)), edges[k]
        assert tuned.energy_estimate(k)[0] == plain.energy_estimate(k)[0]
    for k, s in enumerate(singles):
        assert np.array_equal(tuned.get_field(k), s.get_field()), edges[k]
        assert abs(tuned.energy_estimate(k)[0] - s.energy_estimate()[0]) <= 1e-9 * max(
            1.0, abs(s.energy_estimate()[0]))
    with pytest.raises(lat_mod.LatticeError):
        tuned.autotune(0)


def test_batch_chain_matches_oracle(lat_mod):
    print("[gpu] batch chain vs oracle", flush=True)
    seed = 99
    edges = [(16, 16, 16), (10, 6, 5)]
    b = lat_mod.Batch(edges, "fp32", seed=seed, chain_ids=[4, 9])
    c = workloads.small_neutral(seed=3, L=16, n=10)
    b.set_charges(0, c.xyz, c.q)
    ref = oracle.OracleChain(c.shape, seed=seed, chain=4)
    ref.set_charges(c.xyz, c.q)
    b.run(10, 40, 1)
    ref.sweeps(10)
    s = ref.sweeps(40, 1)
    phi = b.get_field(0).astype(np.float64)
    assert np.abs(phi - ref.phi).max() <= 1e-5 * np.abs(ref.phi).max()
    m, se, M, nb = b.energy_estimate(0)
    assert M == 40 and nb == 40
    scale = np.sum(np.abs(c.q)) ** 2 * np.abs(ref.phi).max() ** 2
    assert abs(m - s[:, 2].mean()) <= 1e-4 * scale
    ref2 = oracle.OracleChain((10, 6, 5), seed=seed, chain=9)
    ref2.sweeps(50)
    assert np.abs(b.get_field(1) - ref2.phi).max() <= 1e-5 * np.abs(ref2.phi).max()


def test_batch_charge_reset_is_per_chain(lat_mod):
    print("[gpu] batch charge reset", flush=True)
    b = lat_mod.Batch([(8, 8, 8), (8, 8, 8)], seed=1)
    for k in range(2):
        b.set_charges(k, [[1, 1, 1], [3, 4, 5]], [1.0, -1.0])
    b.run(0, 20, 5)
    b.set_charges(1, [[2, 2, 2], [5, 5, 5]], [1.0, 1.0])
    b.run(0, 10, 5)
    assert b.energy_estimate(0)[2] == 30
    assert b.energy_estimate(1)[2] == 10


def test_batch_argument_errors(lat_mod):
    print("[gpu] batch errors", flush=True)
    with pytest.raises(lat_mod.LatticeError):
        lat_mod.Batch([(7, 4, 4)])
    b = lat_mod.Batch([(8, 4, 4)])
    with pytest.raises(lat_mod.LatticeError):
        b.set_charges(1, [[0, 0, 0]], [1.0])
    with pytest.raises(lat_mod.LatticeError):
        b.set_charges(0, [[0, 4, 0]], [1.0])
    b.set_charges(0, [[0, 0, 0], [1, 1, 1]], [1.0, -1.0])
    b.run(0, 4, 2)
    with pytest.raises(lat_mod.LatticeError):
        b.run(0, 4, 3)


def test_batched_workload_estimates(lat_mod):
    """The 512-chain workload (edges 24..64, 16..512 charges of N(0,1)
    shifted to neutral): one persistent launch, every chain returns finite
    estimates with the requested bins; chain 0 equals a single lattice."""
    print("[gpu] batched workload", flush=True)
    chains = workloads.batched_chains(seed=0)
    b = lat_mod.Batch([c.shape for c in chains], "fp32", seed=0)
    for k, c in enumerate(chains):
        b.set_charges(k, c.xyz, c.q)
    b.run(20, 200, 20)
    ests = [b.energy_estimate(k) for k in range(len(chains))]
    assert all(np.isfinite(m) and np.isfinite(se) and M == 200 and nb == 10 for m, se, M, nb in ests)
    s = lat_mod.Lattice(chains[0].shape, "fp32", seed=0, chain_id=0)
    s.set_charges(chains[0].xyz, chains[0].q)
    s.thermalise(20)
    s.sweep_and_measure(200, 1, 20)
    assert np.abs(b.get_field(0) - s.get_field()).max() <= 1e-6 * np.abs(s.get_field()).max()
    assert abs(ests[0][0] - s.energy_estimate()[0]) <= 1e-6 * max(1.0, abs(ests[0][0]))


def test_batched_workload_edges_vs_oracle(lat_mod):
    """The 512-chain workload in one launch: the first chain of each edge
    (24, 32, 40, 48, 64) against the oracle chain with the same seed and
    chain id, sweep for sweep (fields within 1e-5 of max |phi|) and sample
    for sample (O within the field tolerance propagated to the sample)."""
    print("[gpu] batched workload edges vs oracle", flush=True)
    chains = workloads.batched_chains(seed=0)
    b = lat_mod.Batch([c.shape for c in chains], "fp32", seed=0)
    for k, c in enumerate(chains):
        b.set_charges(k, c.xyz, c.q)
    b.run(3, 2, 1)
    picks = {}
    for k, c in enumerate(chains):
        picks.setdefault(c.shape[0], k)
    assert sorted(picks) == [24, 32, 40, 48, 64]
    for L, k in sorted(picks.items()):
        c = chains[k]
        ref = oracle.OracleChain(c.shape, seed=0, chain=k)
        ref.set_charges(c.xyz, c.q)
        ref.sweeps(3)
        s = ref.sweeps(2, 1)
        phi = b.get_field(k).astype(np.float64)
        pmax = np.abs(ref.phi).max()
        assert np.abs(phi - ref.phi).max() <= 1e-5 * pmax, L
        m, se, M, nb = b.energy_estimate(k)
        assert M == 2 and nb == 2
        d = 1e-5 * pmax
        dX = d * np.sum(np.abs(c.q))
        dO = 2 * np.abs(s[:, 0]).max() * dX + dX ** 2 + np.sum(c.q ** 2) * (2 * pmax * d + d * d)
        assert abs(m - s[:, 2].mean()) <= dO, (L, m, s[:, 2].mean(), dO)


def test_sharp_energy_batched_16(lat_mod):
    """Unbiasedness of Eq. (nsum2) at a sharp error: 256 independent chains
    of the 16^3 workload (8 charges of +-1, chain ids 1..256) in one batched
    launch, 1e3 thermalisation + 1.5e5 measured sweeps each.  The pooled mean
    (spread of the chains' means over sqrt(256)) lies within 3 sigma of the
    exact lattice energy (dense Cholesky of the 4096 x 4096 Laplacian), and
    sigma is below 2% of |E|."""
    print("[gpu] sharp energy, 256 batched 16^3 chains", flush=True)
    from oracle import exact as ex

    c = workloads.small_neutral(seed=0)
    e_exact = ex.energy_dense(c.shape, c.xyz, c.q)
    n = 256
    b = lat_mod.Batch([c.shape] * n, "fp32", seed=0, chain_ids=list(range(1, n + 1)))
    for k in range(n):
        b.set_charges(k, c.xyz, c.q)
    b.run(1000, 150000, 1000)
    means = np.array([b.energy_estimate(k)[0] for k in range(n)])
    mean, sigma = means.mean(), means.std(ddof=1) / np.sqrt(n)
    print(f"[gpu] pooled {mean:.6f} +- {sigma:.6f}, exact {e_exact:.6f}", flush=True)
    assert sigma < 0.02 * abs(e_exact), (sigma, e_exact)
    assert abs(mean - e_exact) < 3 * sigma, (mean, sigma, e_exact)
