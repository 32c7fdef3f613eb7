"""Pins of the oracle's one-site evaluation used by the large-box parity
checks (CPU only).  ``orc_site_values_f32`` recomputes the heat-bath value
of chosen sites from an FP32 field; it must be the value the oracle's
half-sweep computes before rounding, at every site of either colour,
boundary faces and corners included, and must equal the paper's update
(Eq. phi) written independently here: the neighbour mean with Dirichlet
ghosts (numpy padding) plus the quantile of the site's uniform (scipy's
``ndtri``) over sqrt(6)."""

import numpy as np
import pytest
import scipy.special

import oracle

SHAPES = [(2, 1, 1), (2, 2, 1), (4, 3, 2), (10, 6, 5), (8, 8, 8)]


def _sites_of_colour(shape, c):
    lx, ly, lz = shape
    z, y, x = np.meshgrid(np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    m = ((x + y + z) & 1) == c
    return np.stack([x[m], y[m], z[m]], axis=1).astype(np.int64)


def _neighbour_mean(phi):
    p = np.pad(phi, 1)  # phi = 0 outside the box
    return (p[:-2, 1:-1, 1:-1] + p[2:, 1:-1, 1:-1] + p[1:-1, :-2, 1:-1] + p[1:-1, 2:, 1:-1]
            + p[1:-1, 1:-1, :-2] + p[1:-1, 1:-1, 2:]) / 6.0


@pytest.mark.parametrize("shape", SHAPES)
def test_site_values_equal_halfsweep_values(orc, shape):
    """Every site of both colours: the one-site values rounded to FP32 are
    the oracle half-sweep's stored values, bit for bit, and before rounding
    they are the half-sweep's own site function on the same field."""
    lib = orc.load()
    rng = np.random.default_rng(sum(shape))
    phi32 = rng.standard_normal(shape[::-1]).astype(np.float32)
    for h in (6, 7, 40, 41):
        c = h & 1
        sites = _sites_of_colour(shape, c)
        vals = orc.site_values_f32(phi32, sites, seed=5, chain=3, h=h)
        lx, ly, lz = shape
        direct = np.array([lib.orc_site_value(oracle._ptr(np.ascontiguousarray(phi32, dtype=np.float64)),
                                              lx, ly, lz, int(x), int(y), int(z), 5, 3, h)
                           for x, y, z in sites])
        np.testing.assert_array_equal(vals, direct)
        ch = oracle.OracleChain(shape, "fp32", seed=5, chain=3)
        ch.set_field(phi32)
        ch.halfsweep(h)
        got = ch.phi[sites[:, 2], sites[:, 1], sites[:, 0]]
        np.testing.assert_array_equal(got, vals.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("shape", SHAPES)
def test_site_values_follow_eq_phi(orc, shape):
    """Value = mean of the 6 neighbours (0 beyond the faces) + Phi^-1(r)/sqrt 6,
    with r the site's uniform, against numpy's padded stencil and scipy's
    quantile (which agree with the oracle's to far below this tolerance)."""
    rng = np.random.default_rng(7 + sum(shape))
    phi32 = (3.0 * rng.standard_normal(shape[::-1])).astype(np.float32)
    mean = _neighbour_mean(phi32.astype(np.float64))
    for h in (0, 1, 99):
        sites = _sites_of_colour(shape, h & 1)
        vals = orc.site_values_f32(phi32, sites, seed=11, chain=0, h=h)
        r = np.array([orc.site_uniform(shape, int(x), int(y), int(z), 11, 0, h) for x, y, z in sites])
        want = mean[sites[:, 2], sites[:, 1], sites[:, 0]] + scipy.special.ndtri(r) / np.sqrt(6.0)
        np.testing.assert_allclose(vals, want, rtol=0, atol=1e-13)


def test_site_values_pick_the_right_neighbours(orc):
    """A single non-zero value: only its 6 neighbours (inside the box) move
    by exactly value/6 against an all-zero field."""
    shape = (6, 5, 4)
    lx, ly, lz = shape
    for (x0, y0, z0) in [(0, 0, 0), (5, 4, 3), (2, 2, 1), (3, 0, 2)]:
        phi = np.zeros(shape[::-1], dtype=np.float32)
        phi[z0, y0, x0] = 1.5
        c = (x0 + y0 + z0 + 1) & 1
        sites = _sites_of_colour(shape, c)
        base = orc.site_values_f32(np.zeros_like(phi), sites, seed=2, chain=0, h=c)
        vals = orc.site_values_f32(phi, sites, seed=2, chain=0, h=c)
        d = vals - base
        nbr = np.abs(sites - np.array([x0, y0, z0])).sum(axis=1) == 1
        np.testing.assert_allclose(d[nbr], 0.25, rtol=0, atol=1e-15)
        np.testing.assert_array_equal(d[~nbr], 0.0)
        assert nbr.sum() == sum(1 for dx, dy, dz in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1),
                                                      (0, 0, -1)]
                                if 0 <= x0 + dx < lx and 0 <= y0 + dy < ly and 0 <= z0 + dz < lz)
