"""Pins of the oracle's off-lattice charges (a charge at an arbitrary position
spread over the 8 corners of its lattice cell, the paper's closing remark) and
of its force estimator, against independent definitions: scipy's trilinear
grid interpolator, the on-lattice gather at integer positions, linear fields,
finite differences of the exact energy, and exact Gaussian sampling of the
field."""

import math

import numpy as np
import pytest
import scipy.interpolate

import oracle
from oracle import exact


def _positions(rng, shape, n, margin=0.0):
    hi = np.array(shape, dtype=np.float64) - 1.0
    return rng.uniform(margin, 1.0, size=(n, 3)) * (hi - 2 * margin) + margin


def test_interpolation_matches_scipy_trilinear(orc):
    rng = np.random.default_rng(0)
    shape = (7, 5, 6)
    lx, ly, lz = shape
    phi = rng.standard_normal((lz, ly, lx))
    r = _positions(rng, shape, 200)
    r[:4] = [[0, 0, 0], [lx - 1, ly - 1, lz - 1], [lx - 1, 0, 2.5], [3.25, ly - 1, 0]]  # box corners and faces
    q = rng.standard_normal(200)
    X, Y, phit, grad = oracle.gather_offlattice(phi, r, q)
    interp = scipy.interpolate.RegularGridInterpolator((np.arange(lz), np.arange(ly), np.arange(lx)), phi,
                                                       method="linear")
    want = interp(r[:, ::-1])
    assert np.abs(phit - want).max() < 1e-13
    assert abs(X - float(np.sum(q * want))) < 1e-12
    assert abs(Y - float(np.sum((q * want) ** 2))) < 1e-12
    # gradient: one-sided differences of scipy's interpolant within the cell
    inner = _positions(rng, shape, 50, margin=0.0)
    inner = np.floor(inner) + 0.25 + 0.5 * rng.uniform(size=inner.shape)  # away from cell faces
    inner = np.minimum(inner, np.array(shape) - 1.25)
    _, _, _, g = oracle.gather_offlattice(phi, inner, np.ones(50))
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (interp((inner + e)[:, ::-1]) - interp((inner - e)[:, ::-1])) / (2 * h)
        assert np.abs(g[:, d] - fd).max() < 1e-7, d


def test_integer_positions_reduce_to_site_gather(orc):
    rng = np.random.default_rng(1)
    shape = (6, 4, 5)
    lx, ly, lz = shape
    phi = rng.standard_normal((lz, ly, lx))
    xyz = np.stack([rng.integers(0, lx, 40), rng.integers(0, ly, 40), rng.integers(0, lz, 40)], axis=1)
    xyz[:3] = [[lx - 1, ly - 1, lz - 1], [0, 0, 0], [lx - 1, 0, lz - 1]]  # the clamped top cells
    q = rng.standard_normal(40)
    X, Y, phit, _ = oracle.gather_offlattice(phi, xyz.astype(np.float64), q)
    ch = oracle.OracleChain(shape)
    ch.phi = phi
    ch.set_charges(xyz.astype(np.int32), q)
    X0, Y0 = ch.gather()
    np.testing.assert_array_equal(phit, phi[xyz[:, 2], xyz[:, 1], xyz[:, 0]])
    assert abs(X - X0) < 1e-13 and abs(Y - Y0) < 1e-13


def test_linear_fields_are_interpolated_exactly(orc):
    rng = np.random.default_rng(2)
    shape = (9, 7, 8)
    lx, ly, lz = shape
    a, b, c, d = 0.3, -1.1, 0.7, 2.0
    z, y, x = np.meshgrid(np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    phi = a + b * x + c * y + d * z
    r = _positions(rng, shape, 100)
    _, _, phit, grad = oracle.gather_offlattice(phi, r, np.ones(100))
    assert np.abs(phit - (a + b * r[:, 0] + c * r[:, 1] + d * r[:, 2])).max() < 1e-12
    assert np.abs(grad - np.array([b, c, d])).max() < 1e-12


def test_exact_offlattice_energy_at_sites_is_the_site_energy():
    rng = np.random.default_rng(3)
    shape = (6, 5, 4)
    G = exact.green_dense(shape)
    xyz = np.array([[1, 2, 3], [4, 0, 1], [5, 4, 3], [0, 0, 0], [5, 4, 3]])  # a co-located pair too
    q = rng.standard_normal(5)
    e_site = exact.energy_dense(shape, xyz, q, G)
    e_off = exact.energy_offlattice_dense(shape, xyz.astype(np.float64), q, G)
    assert abs(e_site - e_off) < 1e-12


def test_exact_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    shape = (6, 5, 5)
    G = exact.green_dense(shape)
    r = np.floor(_positions(rng, shape, 4)) + 0.2 + 0.6 * rng.uniform(size=(4, 3))
    r = np.minimum(r, np.array(shape) - 1.2)
    q = np.array([1.0, -0.7, 0.4, 1.3])
    g = exact.grad_offlattice_dense(shape, r, q, G)
    h = 1e-6
    for i in range(4):
        for d in range(3):
            rp, rm = r.copy(), r.copy()
            rp[i, d] += h
            rm[i, d] -= h
            fd = (exact.energy_offlattice_dense(shape, rp, q, G)
                  - exact.energy_offlattice_dense(shape, rm, q, G)) / (2 * h)
            assert abs(g[i, d] - fd) < 1e-7 * max(1.0, abs(fd)), (i, d)


def test_estimators_unbiased_for_exact_gaussian_fields(orc):
    """Fields drawn exactly from N(0, G) (Cholesky): the mean of O equals the
    exact off-lattice energy and the mean of the force sample equals the
    exact dE/dr, within 5 standard errors."""
    rng = np.random.default_rng(5)
    shape = (5, 4, 4)
    lx, ly, lz = shape
    G = exact.green_dense(shape)
    C = np.linalg.cholesky(G)
    r = np.array([[1.3, 1.6, 1.2], [2.7, 1.4, 2.2], [3.1, 2.5, 1.9]])
    q = np.array([1.0, -1.0, 0.6])
    e = exact.energy_offlattice_dense(shape, r, q, G)
    g = exact.grad_offlattice_dense(shape, r, q, G)
    n = 40000
    O = np.empty(n)
    F = np.empty((n, 3, 3))
    Z = rng.standard_normal((C.shape[0], n))
    phis = (C @ Z).T
    for s in range(n):
        phi = phis[s].reshape(lz, ly, lx)
        X, Y, phit, grad = oracle.gather_offlattice(phi, r, q)
        O[s] = X * X - Y
        F[s] = oracle.force_sample(X, phit, grad, q)
    assert abs(O.mean() - e) <= 5 * O.std() / math.sqrt(n)
    err = F.std(axis=0) / math.sqrt(n)
    assert np.all(np.abs(F.mean(axis=0) - g) <= 5 * err + 1e-12)


def test_heat_bath_chain_estimates_offlattice_energy(orc):
    """The oracle's heat-bath chain sampled with off-lattice charges: the mean
    of O after every sweep estimates the exact interpolated energy."""
    shape = (8, 8, 8)
    G = exact.green_dense(shape)
    r = np.array([[2.5, 3.25, 4.0], [4.75, 4.1, 3.3], [3.2, 5.6, 2.4], [5.5, 2.2, 5.1]])
    q = np.array([1.0, 1.0, -1.0, -1.0])
    e = exact.energy_offlattice_dense(shape, r, q, G)
    ch = oracle.OracleChain(shape, seed=17)
    ch.sweeps(200)
    O = []
    for _ in range(20000):
        ch.sweeps(1)
        X, Y, _, _ = oracle.gather_offlattice(ch.phi, r, q)
        O.append(X * X - Y)
    m, se, _, _ = oracle.estimate(np.array(O), 500)
    assert abs(m - e) <= 4 * se, (m, e, se)
