"""Seeded synthetic charge sets for the lattice Coulomb-energy estimator.

This module only places charges on lattice sites; it holds none of the
method's arithmetic (no field, no Green's function, no estimator), so both
the HIP path and the CPU oracle can be fed from it.

The paper measures only synthetic systems: charges put on lattice sites by
rule (a pair moved along the x axis for its two-body test, solid cubes of
N = 8 ... 32768 unit charges for its N-body accuracy test, one charge per
site for its weak-scaling test) on an L^3 box with open boundaries.  The
named workloads below follow that style at the sizes this library is built
and measured for; every array is drawn from ``numpy.random.default_rng``
with a fixed seed, so a (name, seed) pair always gives the same charges.

Coordinates are 0-based ``(x, y, z)`` with ``0 <= x < lx`` etc.; the
paper's 1-based site ``n`` maps to ``n - 1`` here.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ChargeSet",
    "distinct_sites",
    "small_neutral",
    "large_neutral",
    "batched_chains",
    "gaussian_blob",
    "largest_subdomain",
    "pair_scan",
    "solid_cube",
    "WORKLOADS",
]


@dataclass
class ChargeSet:
    """Charges ``q[i]`` on lattice sites ``xyz[i] = (x, y, z)`` of an ``lx*ly*lz`` box."""

    shape: tuple  # (lx, ly, lz)
    xyz: np.ndarray  # int32, (N, 3)
    q: np.ndarray  # float64, (N,)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


def _decode(lin: np.ndarray, lx: int, ly: int) -> np.ndarray:
    x = lin % lx
    y = (lin // lx) % ly
    z = lin // (lx * ly)
    return np.stack([x, y, z], axis=1).astype(np.int32)


def distinct_sites(rng: np.random.Generator, n: int, lo, hi) -> np.ndarray:
    """``n`` distinct sites drawn uniformly from the box ``lo <= (x,y,z) < hi``.

    Draws with replacement and drops repeats (first occurrence wins, in draw
    order) until ``n`` sites are collected; never materialises the box.
    """
    lo = np.asarray(lo, dtype=np.int64)
    hi = np.asarray(hi, dtype=np.int64)
    ext = hi - lo
    vol = int(np.prod(ext))
    if n > vol:
        raise ValueError(f"cannot place {n} distinct sites in a box of {vol}")
    chosen = np.empty(0, dtype=np.int64)
    while chosen.size < n:
        need = n - chosen.size
        draw = rng.integers(0, vol, size=int(need * 1.05) + 16, dtype=np.int64)
        cat = np.concatenate([chosen, draw])
        _, first = np.unique(cat, return_index=True)
        first.sort()
        chosen = cat[first][:n]
    rel = _decode(chosen, int(ext[0]), int(ext[1])).astype(np.int64)
    return (rel + lo[None, :]).astype(np.int32)


def _pm_ones(n_plus: int, n_minus: int, interleave: bool = True) -> np.ndarray:
    if interleave and n_plus == n_minus:
        q = np.empty(n_plus + n_minus)
        q[0::2] = 1.0
        q[1::2] = -1.0
        return q
    return np.concatenate([np.ones(n_plus), -np.ones(n_minus)])


def small_neutral(seed: int = 0, L: int = 16, n: int = 8) -> ChargeSet:
    """Small neutral set: ``n`` charges of +-1 (half each) at distinct interior
    sites (every coordinate in ``[1, L-2]``) of an ``L^3`` box (default 16^3, N=8)."""
    rng = np.random.default_rng(seed)
    xyz = distinct_sites(rng, n, (1, 1, 1), (L - 1, L - 1, L - 1))
    q = _pm_ones(n // 2, n - n // 2, interleave=False)
    return ChargeSet((L, L, L), xyz, q, f"small_neutral_{L}", {"seed": seed})


def large_neutral(seed: int = 0, L: int = 256, n: int = 65536) -> ChargeSet:
    """Large single chain: ``n`` charges of +-1 (neutral) at distinct uniform
    sites of ``L^3``; signs alternate so every even-length prefix (e.g. the
    first 1024) is neutral as well (default 256^3, N=65536)."""
    rng = np.random.default_rng(seed)
    xyz = distinct_sites(rng, n, (0, 0, 0), (L, L, L))
    q = _pm_ones(n // 2, n - n // 2, interleave=True)
    return ChargeSet((L, L, L), xyz, q, f"large_neutral_{L}", {"seed": seed})


def batched_chains(seed: int = 0, n_chains: int = 512, edges=(24, 32, 40, 48, 64),
                   n_lo: int = 16, n_hi: int = 512) -> list:
    """Many independent chains: edge ``L`` uniform over ``edges`` (cubic
    boxes), ``N`` uniform in ``[n_lo, n_hi]``, charges ``N(0,1)`` shifted to
    zero total, distinct sites.  Returns a list of :class:`ChargeSet`."""
    rng = np.random.default_rng(seed)
    out = []
    Ls = rng.choice(np.asarray(edges), size=n_chains)
    Ns = rng.integers(n_lo, n_hi + 1, size=n_chains)
    for k in range(n_chains):
        L = int(Ls[k])
        n = int(Ns[k])
        xyz = distinct_sites(rng, n, (0, 0, 0), (L, L, L))
        q = rng.standard_normal(n)
        q = q - q.mean()
        out.append(ChargeSet((L, L, L), xyz, q, f"chain{k}_{L}", {"seed": seed, "chain": k}))
    return out


def gaussian_blob(seed: int = 0, L: int = 384, n: int = 200_000, sigma: float = 48.0,
                  charge: float = 1.0) -> ChargeSet:
    """Same-sign (gravity-like) set: ``n`` charges ``q = charge`` at distinct
    sites drawn from an isotropic Gaussian of width ``sigma`` sites about the
    box centre ``(L/2, L/2, L/2)``, rounded to the nearest site; draws outside
    the box or on an already-used site are redrawn."""
    rng = np.random.default_rng(seed)
    c = L // 2
    have = np.empty(0, dtype=np.int64)
    while have.size < n:
        need = n - have.size
        pts = np.rint(rng.normal(c, sigma, size=(int(need * 1.1) + 16, 3))).astype(np.int64)
        ok = np.all((pts >= 0) & (pts < L), axis=1)
        pts = pts[ok]
        lin = pts[:, 0] + L * (pts[:, 1] + L * pts[:, 2])
        cat = np.concatenate([have, lin])
        _, first = np.unique(cat, return_index=True)
        first.sort()
        have = cat[first][:n]
    xyz = _decode(have, L, L)
    q = np.full(n, float(charge))
    return ChargeSet((L, L, L), xyz, q, f"gaussian_blob_{L}", {"seed": seed, "sigma": sigma})


def largest_subdomain(seed: int = 0, L: int = 768, n_pm: int = 1_000_000,
                      n_gauss: int = 100_000, gauss_sd: float = 0.5) -> ChargeSet:
    """Largest single-GPU lattice: ``n_pm`` charges of +-1 (half each) plus
    ``n_gauss`` charges drawn from ``N(0, gauss_sd^2)`` (not shifted), all at
    distinct uniform sites of ``L^3`` (default 768^3, 1.1e6 charges)."""
    rng = np.random.default_rng(seed)
    xyz = distinct_sites(rng, n_pm + n_gauss, (0, 0, 0), (L, L, L))
    q = np.concatenate([_pm_ones(n_pm // 2, n_pm - n_pm // 2, interleave=True),
                        rng.normal(0.0, gauss_sd, size=n_gauss)])
    return ChargeSet((L, L, L), xyz, q, f"largest_subdomain_{L}", {"seed": seed})


def pair_scan(L: int = 128, nx: int = 70) -> ChargeSet:
    """Two unit charges: one at the box centre ``(L/2, L/2, L/2)`` (paper's
    1-based centre, 0-based here), the other at ``(nx, L/2, L/2)`` on the
    same x line (the paper's two-body test)."""
    c = L // 2
    xyz = np.array([[c, c, c], [nx, c, c]], dtype=np.int32)
    return ChargeSet((L, L, L), xyz, np.ones(2), f"pair_{L}_{nx}", {})


def solid_cube(L: int = 128, side: int = 2) -> ChargeSet:
    """``side^3`` unit charges filling the cube whose 1-based corners are
    ``L/2 - side/2 + 1`` and ``L/2 + side/2`` on every axis (the paper's
    N-body accuracy test); returned 0-based."""
    lo = L // 2 - side // 2  # 1-based lo minus one
    r = np.arange(lo, lo + side)
    zz, yy, xx = np.meshgrid(r, r, r, indexing="ij")
    xyz = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.int32)
    return ChargeSet((L, L, L), xyz, np.ones(side ** 3), f"cube_{L}_{side}", {})


# Named workloads and their run recipes (sweep counts, storage).  The sizes
# are those the library is built and benchmarked for.
WORKLOADS = {
    "small_neutral_16": dict(make=small_neutral, storage="fp32", therm=1000, meas=10000,
                             bin_size=100, philox_seed=0),
    "large_neutral_256": dict(make=large_neutral, storage="fp32", therm=2000, meas=20000,
                              bin_size=100, philox_seed=0),
    "batched_512": dict(make=batched_chains, storage="fp32", therm=1000, meas=10000,
                        bin_size=100, philox_seed=0),
    "gaussian_blob_384": dict(make=gaussian_blob, storage=("fp32", "bf16", "fp16"), therm=0,
                              meas=10000, bin_size=100, philox_seed=0),
    "largest_subdomain_768": dict(make=largest_subdomain, storage=("fp32", "fp16"), therm=500,
                                  meas=5000, bin_size=100, philox_seed=0),
}
