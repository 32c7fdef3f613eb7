"""Pins of the exact references: the lattice Green's function by independent
routes, its textbook values and its continuum limit (CPU only)."""

import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import exact as ex

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "lattice_green_constants.json")))


def _rand_charges(shape, n, seed):
    rng = np.random.default_rng(seed)
    xyz = np.stack([rng.integers(0, s, n) for s in shape], axis=1)
    return xyz, rng.standard_normal(n)


def test_dense_laplacian_is_the_action_hessian():
    """H_L = 1/2 sum_<m,n> (phi_m - phi_n)^2 with phi = 0 ghosts equals
    1/2 phi^T A phi for the dense -Delta_L (checked on random fields, with
    the pair sum written out bond by bond, ghost bonds included)."""
    shape = (5, 4, 3)
    A = ex.laplacian_dense(shape)
    lx, ly, lz = shape
    rng = np.random.default_rng(0)
    for _ in range(5):
        phi = rng.standard_normal((lz + 2, ly + 2, lx + 2))
        phi[0, :, :] = phi[-1, :, :] = 0
        phi[:, 0, :] = phi[:, -1, :] = 0
        phi[:, :, 0] = phi[:, :, -1] = 0
        H = 0.0
        for ax in range(3):
            d = np.diff(phi, axis=ax)
            H += 0.5 * np.sum(d * d)
        v = phi[1:-1, 1:-1, 1:-1].ravel()
        assert abs(H - 0.5 * v @ A @ v) < 1e-12 * max(1.0, H)
    np.testing.assert_array_equal(ex.laplacian_sparse(shape).toarray(), A)


def test_green_dense_inverts_laplacian():
    shape = (6, 5, 4)
    G = ex.green_dense(shape)
    A = ex.laplacian_dense(shape)
    assert np.abs(A @ G - np.eye(A.shape[0])).max() < 1e-13
    assert np.abs(G - G.T).max() < 1e-15
    assert np.all(G > 0)  # -Delta_L is an M-matrix: its inverse is positive


@pytest.mark.parametrize("shape", [(6, 5, 4), (8, 8, 8), (16, 16, 16)])
def test_dst_matches_cholesky(shape):
    G = ex.green_dense(shape)
    xyz, q = _rand_charges(shape, 12, 1)
    lx, ly, _ = shape
    s = xyz[:, 0] + lx * (xyz[:, 1] + ly * xyz[:, 2])
    ref = float(q @ G[np.ix_(s, s)] @ q)
    assert abs(ex.qGq_dst(shape, xyz, q) - ref) < 1e-12 * abs(ref) + 1e-14
    # diagonal: heat-kernel quadrature and direct mode sum
    d = np.diag(G)[s]
    assert np.abs(ex.green_diag_heat(shape, xyz) - d).max() < 1e-11
    assert np.abs(ex.green_diag_modes(shape, xyz) - d).max() < 1e-13
    assert abs(ex.energy_dst(shape, xyz, q) - ex.energy_dense(shape, xyz, q, G)) < 1e-10


def test_cg_matches_cholesky():
    shape = (8, 7, 6)
    G = ex.green_dense(shape)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(G.shape[0])
    u = ex.solve_cg(shape, b)
    assert np.abs(u - G @ b).max() < 1e-10 * np.abs(G @ b).max()


def test_cg_matches_dst_at_32():
    """Independent of any dense inverse: q^T G q at 32^3 by CG and by DST-I."""
    shape = (32, 32, 32)
    xyz, q = _rand_charges(shape, 40, 3)
    rho = np.zeros(32**3)
    np.add.at(rho, xyz[:, 0] + 32 * (xyz[:, 1] + 32 * xyz[:, 2]), q)
    u = ex.solve_cg(shape, rho)
    assert abs(rho @ u - ex.qGq_dst(shape, xyz, q)) < 1e-9 * abs(rho @ u)


def test_watson_integral():
    """G_inf(0) = W/6 with W Watson's simple-cubic integral (textbook value),
    computed both from the Gamma-function closed form and by integrating the
    Bessel representation numerically."""
    W = GOLD["watson_simple_cubic"]["value"]
    assert abs(ex.watson_closed_form() - W / 6) < 1e-14
    assert abs(ex.green_infinite((0, 0, 0)) - W / 6) < 1e-12


def test_stencil_identity_infinite_lattice():
    """(-Delta_L G)(0) = 1 with cubic symmetry gives 6 G(0) - 6 G(e_x) = 1."""
    assert abs(ex.green_infinite((1, 0, 0)) - (ex.green_infinite((0, 0, 0)) - 1 / 6)) < 1e-12
    # and at a site off the origin: 6 G(n) - sum of its neighbours = 0
    n = (2, 1, 0)
    nb = [(3, 1, 0), (1, 1, 0), (2, 2, 0), (2, 0, 0), (2, 1, 1), (2, 1, -1)]
    val = 6 * ex.green_infinite(n) - sum(ex.green_infinite(m) for m in nb)
    assert abs(val) < 1e-11


def test_coulomb_limit():
    """4 pi r G_inf(r) -> 1 at large r (the continuum Green's function
    1/(4 pi r)); lattice corrections fall off as 1/r^2."""
    c = GOLD["coulomb_limit"]["value"]
    prev = None
    for r in (2, 4, 8, 16):
        ratio = ex.green_infinite((r, 0, 0)) * r / c
        assert 1.0 < ratio < 1.0 + 0.4 / r**2
        if prev is not None:
            assert abs(ratio - 1) < abs(prev - 1)
        prev = ratio
    ratio = ex.green_infinite((10, 10, 10)) * math.sqrt(300) / c
    assert abs(ratio - 1) < 1e-3


def test_dirichlet_centre_converges_to_infinite_lattice():
    """The Dirichlet-box centre value rises to G_inf(0) as the box grows;
    the deficit is the field of the boundary, O(1/L)."""
    ginf = ex.watson_closed_form()
    prev = 0.0
    for L in (9, 17, 33, 65):
        c = L // 2
        g = ex.green_diag_heat((L, L, L), np.array([[c, c, c]]))[0]
        assert prev < g < ginf
        assert ginf - g < 1.5 / (4 * math.pi * (L / 2))
        prev = g


def test_continuum_sum_closed_forms():
    """Eq. (s1) sums ordered pairs: two charges at distance r give
    2 q1 q2 / (4 pi r); three collinear unit charges at spacing d give
    2 (1/d + 1/d + 1/(2d)) / (4 pi)."""
    assert abs(ex.energy_continuum([[0, 0, 0], [3, 4, 0]], [2.0, -1.5]) - 2 * (-3.0) / (4 * math.pi * 5)) < 1e-15
    d = 3.0
    e = ex.energy_continuum([[0, 0, 0], [d, 0, 0], [2 * d, 0, 0]], [1, 1, 1])
    assert abs(e - 2 * (2 / d + 1 / (2 * d)) / (4 * math.pi)) < 1e-15


def test_lattice_pair_energy_approaches_continuum():
    """A unit pair at distance 6 in the centre of an L^3 box: E_lat rises to
    the infinite-lattice value 2 G_inf(6) with a boundary deficit that halves
    each time L doubles (the open-boundary effect), and 2 G_inf(6) is within
    1% of the continuum Eq. (s1)."""
    r = 6
    e_inf = 2 * ex.green_infinite((r, 0, 0))
    e_cont = ex.energy_continuum([[0, 0, 0], [r, 0, 0]], [1.0, 1.0])
    assert 0 < e_inf / e_cont - 1 < 0.01
    deficits = []
    for L in (32, 64, 128, 256):
        c = L // 2
        xyz = np.array([[c - r // 2, c, c], [c + r // 2, c, c]])
        deficits.append(e_inf - ex.energy_dst((L, L, L), xyz, [1.0, 1.0]))
    assert all(d > 0 for d in deficits)
    for a, b in zip(deficits[:-1], deficits[1:]):
        assert 1.8 < a / b < 2.4


def test_energy_pair_sum_definition():
    """energy_dense sums q_i q_j G_ij over ordered pairs i != j, including
    co-located charges (two charges on one site pair through G(n, n))."""
    shape = (4, 4, 4)
    G = ex.green_dense(shape)
    xyz = np.array([[1, 1, 1], [1, 1, 1], [2, 3, 0]])
    q = np.array([0.5, -2.0, 1.5])
    i0, i2 = 1 + 4 * (1 + 4 * 1), 2 + 4 * (3 + 4 * 0)
    ref = 2 * (0.5 * -2.0 * G[i0, i0] + 0.5 * 1.5 * G[i0, i2] + -2.0 * 1.5 * G[i0, i2])
    assert abs(ex.energy_dense(shape, xyz, q, G) - ref) < 1e-15
    assert abs(ex.energy_dst(shape, xyz, q) - ref) < 1e-12


def test_c2_subset_energy_by_cg_per_charge():
    """The 256^3 exact reference (DST-I for q^T G q, heat-kernel quadrature
    for the diagonal) against FP64 conjugate gradients per charge, with no
    transform: a 3-charge subset of the first 1,024 charges of the 65,536-
    charge workload, chosen as the closest pair and the charge nearest its
    midpoint so that the pair terms are not lost next to the diagonal.  Two
    CG columns give every pair of the three (about 50 s on 8 cores)."""
    from paper_1403_0711_amd import workloads

    c = workloads.large_neutral()
    x = c.xyz[:1024].astype(np.int64)
    q = c.q[:1024]
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.iinfo(np.int64).max)
    a, b = np.unravel_index(np.argmin(d2), d2.shape)
    dm = ((x - (x[a] + x[b]) / 2.0) ** 2).sum(-1)
    dm[[a, b]] = np.inf
    k = int(np.argmin(dm))
    ua = oracle.green_column_cg(c.shape, x[a])
    ub = oracle.green_column_cg(c.shape, x[b])

    def g(u, s):
        return u[s[2], s[1], s[0]]

    Gab, Gac, Gbc = g(ua, x[b]), g(ua, x[k]), g(ub, x[k])
    assert abs(g(ub, x[a]) - Gab) <= 1e-12 * Gab  # G is symmetric
    E_cg = 2.0 * (q[a] * q[b] * Gab + q[a] * q[k] * Gac + q[b] * q[k] * Gbc)
    sel = [a, b, k]
    E_dst = ex.energy_dst(c.shape, x[sel], q[sel])
    assert abs(E_cg - E_dst) <= 1e-9 * abs(E_dst), (E_cg, E_dst)
    # the columns' diagonal entries against the heat-kernel quadrature
    h = ex.green_diag_heat(c.shape, x[[a, b]])
    assert abs(g(ua, x[a]) - h[0]) <= 1e-12 * h[0]
    assert abs(g(ub, x[b]) - h[1]) <= 1e-12 * h[1]
