"""CPU oracle for the heat-bath lattice Coulomb-energy estimator.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library.

Two parts:

* :class:`OracleChain` (backed by ``heatbath_oracle.c``): the same red-black
  heat bath, with the same Philox streams, in plain FP64 loops; it pins the
  GPU chain sweep by sweep.
* :mod:`oracle.exact`: the exact lattice energy the chain estimates,
  E_lat = sum_{i != j} q_i q_j G(n_i, n_j) with G = (-Delta_L)^{-1} on the
  Dirichlet box, plus the continuum sum (the paper's Eq. s1).

The estimator (the paper's Eq. nsum2) is the sample mean of
O = (sum_i q_i phi_i)^2 - sum_i (q_i phi_i)^2; its error bar is taken from
bins of consecutive samples.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = ["OracleChain", "load", "philox4x32_10", "inv_norm_cdf", "round_storage",
           "round_storage_sr_mean", "site_uniform", "site_word", "noise_grid", "estimate", "gather_offlattice", "force_sample", "STORAGE"]

# storage formats: 16-bit values rounded to nearest even (bf16, fp16) or
# stochastically with the 8 low bits of each site's Philox word (bf16sr, fp16sr)
STORAGE = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16sr": 3, "fp16sr": 4}
_GRID_OF = {0: 0, 1: 1, 2: 2, 3: 1, 4: 2}  # the round-to-nearest format of the same grid

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def load() -> ctypes.CDLL:
    """Load ``liboracle.so``, building it first if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build_oracle import build

        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_philox4x32_10.argtypes = [_p, _p, _p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_norm_cdf.argtypes = [_d]
    lib.orc_norm_cdf.restype = _d
    lib.orc_inv_norm_cdf.argtypes = [_d]
    lib.orc_inv_norm_cdf.restype = _d
    lib.orc_round_storage.argtypes = [_d, ctypes.c_int]
    lib.orc_round_storage.restype = _d
    lib.orc_site_uniform.argtypes = [_i64, _i64, _i64, _i64, _i64, _u64, _u32, _u32]
    lib.orc_site_uniform.restype = _d
    lib.orc_site_word.argtypes = [_i64, _i64, _i64, _i64, _i64, _u64, _u32, _u32]
    lib.orc_site_word.restype = _u32
    lib.orc_round_storage_sr.argtypes = [_d, ctypes.c_int, _u32]
    lib.orc_round_storage_sr.restype = _d
    lib.orc_round_storage_sr_mean.argtypes = [_p, _i64, ctypes.c_int, _p]
    lib.orc_round_storage_sr_mean.restype = None
    lib.orc_site_value.argtypes = [_p, _i64, _i64, _i64, _i64, _i64, _i64, _u64, _u32, _u32]
    lib.orc_site_value.restype = _d
    lib.orc_halfsweep.argtypes = [_p, _i64, _i64, _i64, ctypes.c_int, _u64, _u32, _u32]
    lib.orc_halfsweep.restype = None
    lib.orc_gather.argtypes = [_p, _i64, _i64, _i64, _i64, _p, _p, _p]
    lib.orc_gather.restype = None
    lib.orc_gather_offlattice.argtypes = [_p, _i64, _i64, _i64, _i64, _p, _p, _p, _p, _p]
    lib.orc_gather_offlattice.restype = None
    lib.orc_run.argtypes = [_p, _i64, _i64, _i64, ctypes.c_int, _u64, _u32, _i64, _i64, _i64,
                            _i64, _p, _p, _p]
    lib.orc_run.restype = _i64
    lib.orc_site_values_f32.argtypes = [_p, _i64, _i64, _i64, _i64, _p, _u64, _u32, _u32, _p]
    lib.orc_site_values_f32.restype = None
    lib.orc_noise_grid.argtypes = [_i64, _i64, _p]
    lib.orc_noise_grid.restype = None
    lib.orc_cg_laplacian.argtypes = [_i64, _i64, _i64, _p, _p, _d, _i64]
    lib.orc_cg_laplacian.restype = _i64
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter and 2-word key (uint32 each)."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def inv_norm_cdf(r: float) -> float:
    """Standard-normal quantile Phi^{-1}(r), FP64."""
    return load().orc_inv_norm_cdf(float(r))


def round_storage(v: float, storage: str, u8=None) -> float:
    """An FP64 value rounded to the storage format: to nearest even, or for
    the stochastic formats with random bits ``u8`` (0..255; without them the
    nearest-even rounding of the same grid, which field uploads use)."""
    code = STORAGE[storage]
    if code >= 3 and u8 is not None:
        return load().orc_round_storage_sr(float(v), code, int(u8) & 0xFF)
    return load().orc_round_storage(float(v), _GRID_OF[code])


def round_storage_sr_mean(v: np.ndarray, storage: str) -> np.ndarray:
    """For each FP64 value, the mean of its stochastic roundings (format
    ``bf16sr`` or ``fp16sr``) over the 256 values of the random byte."""
    x = np.ascontiguousarray(v, dtype=np.float64).ravel()
    out = np.empty_like(x)
    load().orc_round_storage_sr_mean(_ptr(x), x.size, STORAGE[storage], _ptr(out))
    return out


def site_uniform(shape, x, y, z, seed, chain, h) -> float:
    lx, ly, _ = shape
    return load().orc_site_uniform(lx, ly, x, y, z, seed, chain, h)


def site_word(shape, x, y, z, seed, chain, h) -> int:
    """The 32-bit Philox word of a site in half-sweep h (its uniform is
    word >> 8, its stochastic-rounding bits word & 0xFF)."""
    lx, ly, _ = shape
    return int(load().orc_site_word(lx, ly, x, y, z, seed, chain, h))


class OracleChain:
    """One heat-bath chain on an ``lx*ly*lz`` Dirichlet box, field in FP64
    (each value exactly representable in the storage format), natural order
    ``phi[z, y, x]``.  The sweep counter ``t`` counts all sweeps since
    creation and keys the random stream, as in the HIP library."""

    def __init__(self, shape, storage: str = "fp32", seed: int = 0, chain: int = 0):
        self.lib = load()
        self.shape = tuple(int(s) for s in shape)
        lx, ly, lz = self.shape
        self.storage = storage
        self.seed = int(seed)
        self.chain = int(chain)
        self.phi = np.zeros((lz, ly, lx), dtype=np.float64)
        self.t = 0
        self.xyz = np.zeros((0, 3), dtype=np.int32)
        self.q = np.zeros(0, dtype=np.float64)
        self.samples = np.zeros((0, 3), dtype=np.float64)

    def set_charges(self, xyz, q):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
        self.q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)

    def set_field(self, phi):
        v = np.asarray(phi, dtype=np.float64).reshape(self.phi.shape)
        if self.storage == "fp32":
            self.phi = v.astype(np.float32).astype(np.float64)
        else:
            f = np.vectorize(lambda a: round_storage(a, self.storage))
            self.phi = f(v).astype(np.float64)

    def halfsweep(self, h: int):
        lx, ly, lz = self.shape
        self.lib.orc_halfsweep(_ptr(self.phi), lx, ly, lz, STORAGE[self.storage], self.seed,
                               self.chain, int(h))

    def sweeps(self, n: int, measure_every: int = 0) -> np.ndarray:
        """``n`` sweeps; returns the (X, Y, O) samples taken (and keeps them)."""
        lx, ly, lz = self.shape
        n = int(n)
        nm = n // measure_every if measure_every > 0 else 0
        out = np.zeros((max(nm, 1), 3), dtype=np.float64)
        m = self.lib.orc_run(_ptr(self.phi), lx, ly, lz, STORAGE[self.storage], self.seed,
                             self.chain, self.t, n, int(measure_every), self.q.shape[0],
                             _ptr(self.xyz), _ptr(self.q), _ptr(out))
        self.t += n
        out = out[:m]
        self.samples = np.concatenate([self.samples, out])
        return out

    def gather(self):
        lx, ly, lz = self.shape
        out = np.zeros(2, dtype=np.float64)
        self.lib.orc_gather(_ptr(self.phi), lx, ly, lz, self.q.shape[0], _ptr(self.xyz),
                            _ptr(self.q), _ptr(out))
        return float(out[0]), float(out[1])


def gather_offlattice(phi: np.ndarray, r, q):
    """Off-lattice charges on a field ``phi[z, y, x]`` (FP64): trilinear
    interpolation from the 8 corners of each charge's cell.  Returns
    ``(X, Y, phit, grad)``: X = sum q phi~, Y = sum (q phi~)^2, phi~ at each
    charge and its gradient (n x 3)."""
    lz, ly, lx = phi.shape
    f = np.ascontiguousarray(phi, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    out = np.zeros(2)
    phit = np.zeros(q.shape[0])
    grad = np.zeros((q.shape[0], 3))
    load().orc_gather_offlattice(_ptr(f), lx, ly, lz, q.shape[0], _ptr(r), _ptr(q), _ptr(out), _ptr(phit),
                                 _ptr(grad))
    return float(out[0]), float(out[1]), phit, grad


def force_sample(X: float, phit: np.ndarray, grad: np.ndarray, q) -> np.ndarray:
    """One sample of dE/dr_i for off-lattice charges (n x 3): E is the mean of
    O = X^2 - Y with X = sum q_j phi~_j and Y = sum (q_j phi~_j)^2, so
    dO/dr_i = 2 q_i grad phi~_i (X - q_i phi~_i).  E sums ordered pairs (the
    paper's Eq. s1), twice the physical pair energy: the physical force on
    charge i is -(1/2) dE/dr_i."""
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    return 2.0 * (q * (X - q * phit))[:, None] * grad


def site_values_f32(phi32: np.ndarray, sites: np.ndarray, seed: int, chain: int, h: int) -> np.ndarray:
    """Heat-bath values (FP64, before rounding) of the listed ``(x,y,z)``
    sites, all of colour ``h & 1``, computed from an FP32 field ``phi[z,y,x]``."""
    lz, ly, lx = phi32.shape
    f = np.ascontiguousarray(phi32, dtype=np.float32)
    s = np.ascontiguousarray(sites, dtype=np.int64).reshape(-1, 3)
    out = np.zeros(s.shape[0], dtype=np.float64)
    load().orc_site_values_f32(_ptr(f), lx, ly, lz, s.shape[0], _ptr(s), int(seed), int(chain),
                               int(h), _ptr(out))
    return out


def noise_grid(k_first: int, n: int) -> np.ndarray:
    """Heat-bath noise Phi^{-1}(r)/sqrt(6) (FP64) at the grid points
    k_first .. k_first + n - 1 of r = (k + 1/2) 2^-24."""
    out = np.zeros(int(n), dtype=np.float64)
    load().orc_noise_grid(int(k_first), int(n), _ptr(out))
    return out


def green_column_cg(shape, site, rtol: float = 1e-13, maxit: int = 100000) -> np.ndarray:
    """Column G(., n) of the lattice propagator G = (-Delta_L)^{-1} (Dirichlet
    box, the Hessian of the paper's discretised action) for the site n =
    (x, y, z): the solution of -Delta_L u = e_n by plain FP64 conjugate
    gradients; array order (z, y, x)."""
    lx, ly, lz = (int(v) for v in shape)
    b = np.zeros((lz, ly, lx))
    b[site[2], site[1], site[0]] = 1.0
    u = np.empty_like(b)
    it = load().orc_cg_laplacian(lx, ly, lz, _ptr(b), _ptr(u), float(rtol), int(maxit))
    if it < 0:
        raise RuntimeError(f"CG failed ({it})")
    return u


def estimate(O: np.ndarray, bin_size: int):
    """Sample mean of O (the paper's Eq. nsum2, summed exactly with fsum) and
    its binned standard error: full bins of ``bin_size`` consecutive samples,
    stderr = sqrt(sum_b (mean_b - mean)^2 / (n_b (n_b - 1))).  A trailing
    partial bin enters the mean, not the error."""
    O = np.asarray(O, dtype=np.float64)
    M = O.shape[0]
    mean = math.fsum(O.tolist()) / M if M else 0.0
    nb = M // bin_size
    if nb < 2:
        return mean, float("nan"), M, nb
    bm = np.array([math.fsum(O[b * bin_size:(b + 1) * bin_size].tolist()) / bin_size
                   for b in range(nb)])
    mb = math.fsum(bm.tolist()) / nb
    se = math.sqrt(math.fsum(((bm - mb) ** 2).tolist()) / (nb * (nb - 1)))
    return mean, se, M, nb
