"""Python binding of the C ABI in ``include/lattice_coulomb.h`` (ctypes).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch supplies device memory (its caching allocator, through the
ABI's allocator callbacks) and the stream (the current torch stream).  The
library must have been built (``python -m paper_1403_0711_amd.build_lib``);
nothing here falls back to another implementation.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Lattice", "Batch", "LatticeError", "load_library", "STORAGE", "VARIANT"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "liblatcoul.so")

# field storage formats (bf16sr and fp16sr round stochastically with the low
# byte of each site's Philox word)
STORAGE = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16sr": 3, "fp16sr": 4}
VARIANT = {"auto": 0, "quad": 1, "generic": 2, "zslab": 3, "fused": 4, "resident": 5, "stream": 6,
           "blocked": 7}
ERR_NAMES = {1: "LAT_ERR_ARG", 2: "LAT_ERR_STATE", 3: "LAT_ERR_ALLOC", 4: "LAT_ERR_DEVICE"}

_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_int = ctypes.c_int
_p = ctypes.c_void_p
_pd = ctypes.POINTER(ctypes.c_double)
_pi64 = ctypes.POINTER(ctypes.c_int64)

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class LatAllocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", ALLOC_FN), ("release", RELEASE_FN)]


class LatticeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library() -> ctypes.CDLL:
    """Load ``liblatcoul.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1403_0711_amd.build_lib` (or __graft_entry__.build())")
    # PyTorch (which provides the device memory and streams) brings its own
    # HIP runtime: load it and let it find the devices before this library's
    # HIP calls, whatever the caller imported first.
    import torch

    torch.cuda.is_available()
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "lattice_create": (_int, [_i64, _i64, _i64, _int, _u64, _u32, _p, _p, _p]),
        "set_charges": (_int, [_p, _i64, _p, _p]),
        "thermalise": (_int, [_p, _i64]),
        "sweep_and_measure": (_int, [_p, _i64, _i64, _i64]),
        "sweep_and_measure_noalloc": (_int, [_p, _i64, _i64, _i64]),
        "energy_estimate": (_int, [_p, _pd, _pd, _pi64, _pi64]),
        "lattice_set_charge_sets": (_int, [_p, _i64, _p, _p, _p]),
        "lattice_energy_estimate_set": (_int, [_p, _i64, _pd, _pd, _pi64, _pi64]),
        "lattice_set_offlattice_charges": (_int, [_p, _i64, _p, _p, _int]),
        "lattice_force_estimate": (_int, [_p, _p, _p, _pi64]),
        "lattice_destroy": (None, [_p]),
        "lattice_last_error": (ctypes.c_char_p, []),
        "lattice_sweep_count": (_int, [_p, _pi64]),
        "lattice_set_variant": (_int, [_p, _int]),
        "lattice_set_tuning": (_int, [_p, _i64, _int, _int]),
        "lattice_use_graphs": (_int, [_p, _int]),
        "lattice_get_tuning": (_int, [_p, ctypes.POINTER(_int), _pi64, ctypes.POINTER(_int), ctypes.POINTER(_int)]),
        "lattice_get_sample_path": (_int, [_p, ctypes.POINTER(_int)]),
        "lattice_get_gather_parts": (_int, [_p, ctypes.POINTER(_int), ctypes.POINTER(_int)]),
        "lattice_autotune": (_int, [_p, _i64, ctypes.POINTER(_int), _pi64, ctypes.POINTER(_int),
                                    ctypes.POINTER(_int), _pd]),
        "lattice_get_field": (_int, [_p, _p]),
        "lattice_set_field": (_int, [_p, _p]),
        "lattice_last_measure": (_int, [_p, _pd, _pd]),
        "lattice_noise_values": (_int, [_i64, _i64, _p, _p]),
        "lattice_get_state": (_int, [_p, _pi64, _pi64, _p, _i64, _pi64]),
        "lattice_set_state": (_int, [_p, _i64, _i64, _i64, _p, _i64]),
        "batch_create": (_int, [_i64, _p, _p, _int, _u64, _p, _p, _p]),
        "batch_set_charges": (_int, [_p, _i64, _i64, _p, _p]),
        "batch_run": (_int, [_p, _i64, _i64, _i64]),
        "batch_autotune": (_int, [_p, _i64, _pi64]),
        "batch_energy_estimate": (_int, [_p, _i64, _pd, _pd, _pi64, _pi64]),
        "batch_get_field": (_int, [_p, _i64, _p]),
        "batch_destroy": (None, [_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise LatticeError(rc, _lib.lattice_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class _TorchMemory:
    """Allocator callbacks backed by torch's caching allocator on one device
    and stream (kept alive as long as the owning handle)."""

    def __init__(self, device, stream):
        import torch

        self.torch = torch
        self.device = device
        self.stream = stream

        self.n_alloc = 0  # allocator calls made through this handle's callbacks

        def _alloc(ctx, nbytes):
            self.n_alloc += 1
            try:
                return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:  # out of memory -> NULL -> LAT_ERR_ALLOC
                return None

        def _release(ctx, ptr):
            try:
                self.torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass

        self._alloc = ALLOC_FN(_alloc)
        self._release = RELEASE_FN(_release)
        self.struct = LatAllocator(None, self._alloc, self._release)


def _device_and_stream(device, stream):
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the lattice estimator runs on the GPU only")
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else int(device))
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    return dev, stream


def noise_values(k_first: int, n: int, device=None):
    """The device's heat-bath noise erfinv(2r - 1)/sqrt(3) at the grid points
    k_first .. k_first + n - 1 of r = (k + 1/2) 2^-24 (test hook): a float32
    numpy array of n values."""
    import torch

    load_library()
    dev, stream = _device_and_stream(device, None)
    out = torch.empty(int(n), dtype=torch.float32, device=dev)
    _check(_lib.lattice_noise_values(int(k_first), int(n), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(stream.cuda_stream)))
    return out.cpu().numpy()


class Lattice:
    """One heat-bath chain on an ``lx*ly*lz`` Dirichlet box (see the header
    for the exact method).  ``shape = (lx, ly, lz)``; fields are returned as
    ``phi[z, y, x]`` float32 arrays."""

    def __init__(self, shape, storage: str = "fp32", seed: int = 0, chain_id: int = 0,
                 device=None, stream=None, allocator: str = "torch"):
        import torch

        self.lib = load_library()
        self.shape = tuple(int(s) for s in shape)
        self.storage = storage
        self.device, self.stream = _device_and_stream(device, stream)
        self._mem = _TorchMemory(self.device, self.stream) if allocator == "torch" else None
        alloc_ptr = ctypes.cast(ctypes.pointer(self._mem.struct), ctypes.c_void_p) if self._mem else None
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.lattice_create(*self.shape, STORAGE[storage], int(seed), int(chain_id),
                                           alloc_ptr, ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(h)))
        self.h = h
        self.n_sets = 1  # charge sets measured per sweep
        self.n_offlattice = 0

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            import torch

            with torch.cuda.device(self.device):
                self.lib.lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _call(self, fn, *args):
        import torch

        with torch.cuda.device(self.device):
            _check(fn(self.h, *args))

    # -- the five calls of the method ------------------------------------
    def set_charges(self, xyz, q):
        xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        if xyz.shape[0] != q.shape[0]:
            raise ValueError("xyz and q differ in length")
        self._call(self.lib.set_charges, q.shape[0], _ptr(xyz), _ptr(q))
        self.n_sets = 1

    def set_charge_sets(self, sets):
        """Several charge sets ``[(xyz, q), ...]`` measured on one field
        chain: every measured sweep takes one sample per set."""
        xs, qs = [], []
        for xyz, q in sets:
            xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
            q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
            if xyz.shape[0] != q.shape[0]:
                raise ValueError("xyz and q differ in length")
            xs.append(xyz)
            qs.append(q)
        counts = np.array([q.shape[0] for q in qs], dtype=np.int64)
        xyz = np.ascontiguousarray(np.concatenate(xs) if xs else np.zeros((0, 3), np.int32), dtype=np.int32)
        q = np.ascontiguousarray(np.concatenate(qs) if qs else np.zeros(0), dtype=np.float64)
        self._call(self.lib.lattice_set_charge_sets, len(counts), _ptr(counts), _ptr(xyz), _ptr(q))
        self.n_sets = len(counts)
    def set_offlattice_charges(self, r, q, forces: bool = False):
        """Charges at real positions ``r`` (n x 3, lattice units), each spread
        over the 8 corners of its cell; with ``forces``, also estimate
        dE/dr per charge (``force_estimate``)."""
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1, 3)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        if r.shape[0] != q.shape[0]:
            raise ValueError("r and q differ in length")
        self._call(self.lib.lattice_set_offlattice_charges, q.shape[0], _ptr(r), _ptr(q), 1 if forces else 0)
        self.n_sets = 1
        self.n_offlattice = q.shape[0]

    def force_estimate(self):
        """Returns ``(dE_dr, stderr, n_samples)`` with arrays (n, 3); the
        physical force is -dE_dr / 2 (E sums ordered pairs)."""
        n = self.n_offlattice
        g = np.zeros((max(n, 1), 3))
        se = np.zeros((max(n, 1), 3))
        m = ctypes.c_int64()
        self._call(self.lib.lattice_force_estimate, _ptr(g), _ptr(se), ctypes.byref(m))
        return g[:n], se[:n], m.value

    def thermalise(self, n_sweeps: int):
        self._call(self.lib.thermalise, int(n_sweeps))

    def sweep_and_measure(self, n_sweeps: int, measure_every: int = 1, bin_size: int = 100):
        self._call(self.lib.sweep_and_measure, int(n_sweeps), int(measure_every), int(bin_size))

    def sweep_and_measure_noalloc(self, n_sweeps: int, measure_every: int = 1, bin_size: int = 100):
        """As ``sweep_and_measure``, allocating nothing (bins must have room)."""
        self._call(self.lib.sweep_and_measure_noalloc, int(n_sweeps), int(measure_every), int(bin_size))

    def energy_estimate(self, allow_few_bins: bool = False, charge_set: int = 0):
        """Returns ``(mean, stderr, n_samples, n_bins)`` of one charge set."""
        import torch

        m, s = ctypes.c_double(), ctypes.c_double()
        n, nb = ctypes.c_int64(), ctypes.c_int64()
        with torch.cuda.device(self.device):
            rc = self.lib.lattice_energy_estimate_set(self.h, int(charge_set), ctypes.byref(m), ctypes.byref(s),
                                                      ctypes.byref(n), ctypes.byref(nb))
        if rc != 0 and not (allow_few_bins and rc == 2 and nb.value < 2):
            _check(rc)
        return m.value, s.value, n.value, nb.value

    # -- hooks -----------------------------------------------------------
    @property
    def sweeps(self) -> int:
        v = ctypes.c_int64()
        self._call(self.lib.lattice_sweep_count, ctypes.byref(v))
        return v.value

    def set_variant(self, name: str):
        self._call(self.lib.lattice_set_variant, VARIANT[name])

    def set_tuning(self, planes: int = 0, tile: int = -1, xcd_order=None):
        """Slab-kernel tuning: planes per workgroup, tile configuration, XCD
        order (0 / -1 / None: library defaults)."""
        x = -1 if xcd_order is None else int(xcd_order)
        self._call(self.lib.lattice_set_tuning, int(planes), int(tile), x)

    def use_graphs(self, mode: int = 1):
        """0: launch by launch; 1: hipGraph chunks for boxes up to 2^24 sites; 2: always."""
        self._call(self.lib.lattice_use_graphs, int(mode))

    def tuning(self) -> dict:
        """The configuration the next sweep runs (library choices resolved)."""
        v, t, x = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        pl = ctypes.c_int64()
        self._call(self.lib.lattice_get_tuning, ctypes.byref(v), ctypes.byref(pl), ctypes.byref(t), ctypes.byref(x))
        names = {val: key for key, val in VARIANT.items()}
        return {"variant": names.get(v.value, v.value), "planes": pl.value, "tile": t.value,
                "xcd_order": int(x.value)}

    def sample_path(self) -> str:
        """How the samples of the last sweep_and_measure were gathered:
        "fused" (inside the streaming sweep kernel) or "separate"."""
        f = ctypes.c_int()
        self._call(self.lib.lattice_get_sample_path, ctypes.byref(f))
        return "fused" if f.value else "separate"

    def gather_parts(self) -> tuple:
        """(parts, entries per part) of the blocked sweep's staged charge
        lists; (0, 0) when samples are not gathered inside that kernel."""
        p, e = ctypes.c_int(), ctypes.c_int()
        self._call(self.lib.lattice_get_gather_parts, ctypes.byref(p), ctypes.byref(e))
        return p.value, e.value

    def autotune(self, reps: int = 5) -> dict:
        """Time the sweep kernels on scratch memory and keep the fastest."""
        v, t, x = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        pl, ms = ctypes.c_int64(), ctypes.c_double()
        self._call(self.lib.lattice_autotune, int(reps), ctypes.byref(v), ctypes.byref(pl), ctypes.byref(t),
                   ctypes.byref(x), ctypes.byref(ms))
        names = {val: key for key, val in VARIANT.items()}
        return {"variant": names.get(v.value, v.value), "planes": pl.value, "tile": t.value,
                "xcd_order": int(x.value), "ms_per_sweep": ms.value}

    def get_field(self) -> np.ndarray:
        lx, ly, lz = self.shape
        out = np.empty((lz, ly, lx), dtype=np.float32)
        self._call(self.lib.lattice_get_field, _ptr(out))
        return out

    def set_field(self, phi):
        lx, ly, lz = self.shape
        a = np.ascontiguousarray(phi, dtype=np.float32).reshape(lz, ly, lx)
        self._call(self.lib.lattice_set_field, _ptr(a))

    def last_measure(self):
        X, Y = ctypes.c_double(), ctypes.c_double()
        self._call(self.lib.lattice_last_measure, ctypes.byref(X), ctypes.byref(Y))
        return X.value, Y.value

    def get_state(self):
        """Returns ``(sweep_counter, n_samples, bins)``: bins (n, 2) for one
        charge set, (n_sets, n, 2) for several."""
        t, n, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._call(self.lib.lattice_get_state, ctypes.byref(t), ctypes.byref(n), None, 0, ctypes.byref(nb))
        k = self.n_sets
        bins = np.zeros((k, max(nb.value, 1), 2), dtype=np.float64)
        self._call(self.lib.lattice_get_state, ctypes.byref(t), ctypes.byref(n), _ptr(bins), k * nb.value,
                   ctypes.byref(nb))
        bins = np.ascontiguousarray(bins[:, :nb.value])
        return t.value, n.value, (bins[0] if k == 1 else bins)

    def set_state(self, sweep_counter: int, n_samples: int, bin_size: int, bins):
        """Restore a checkpoint of ``get_state`` (charge sets placed first)."""
        b = np.ascontiguousarray(bins, dtype=np.float64).reshape(self.n_sets, -1, 2)
        self._call(self.lib.lattice_set_state, int(sweep_counter), int(n_samples), int(bin_size),
                   _ptr(b), b.shape[1])


class Batch:
    """Independent chains on boxes of uneven size, run in one persistent
    launch.  ``edges`` is a list of ``(lx, ly, lz)``."""

    def __init__(self, edges, storage: str = "fp32", seed: int = 0, chain_ids=None, device=None,
                 stream=None, allocator: str = "torch"):
        import torch

        self.lib = load_library()
        self.edges = [tuple(int(v) for v in e) for e in edges]
        self.device, self.stream = _device_and_stream(device, stream)
        self._mem = _TorchMemory(self.device, self.stream) if allocator == "torch" else None
        alloc_ptr = ctypes.cast(ctypes.pointer(self._mem.struct), ctypes.c_void_p) if self._mem else None
        e = np.ascontiguousarray(self.edges, dtype=np.int64).reshape(-1, 3)
        ids = None
        if chain_ids is not None:
            ids = np.ascontiguousarray(chain_ids, dtype=np.uint32)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.batch_create(e.shape[0], _ptr(e), _ptr(ids) if ids is not None else None,
                                         STORAGE[storage], int(seed), alloc_ptr,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            import torch

            with torch.cuda.device(self.device):
                self.lib.batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, *args):
        import torch

        with torch.cuda.device(self.device):
            _check(fn(self.h, *args))

    def set_charges(self, chain: int, xyz, q):
        xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        self._call(self.lib.batch_set_charges, int(chain), q.shape[0], _ptr(xyz), _ptr(q))

    def run(self, n_therm: int, n_meas: int, bin_size: int = 100):
        self._call(self.lib.batch_run, int(n_therm), int(n_meas), int(bin_size))

    def autotune(self, reps: int = 5) -> int:
        """Choose the LDS-ring or memory half-sweep per box by timing scratch
        batches; returns the number of chains that will use the ring."""
        n = ctypes.c_int64()
        self._call(self.lib.batch_autotune, int(reps), ctypes.byref(n))
        return n.value

    def energy_estimate(self, chain: int):
        m, s = ctypes.c_double(), ctypes.c_double()
        n, nb = ctypes.c_int64(), ctypes.c_int64()
        self._call(self.lib.batch_energy_estimate, int(chain), ctypes.byref(m), ctypes.byref(s),
                   ctypes.byref(n), ctypes.byref(nb))
        return m.value, s.value, n.value, nb.value

    def get_field(self, chain: int) -> np.ndarray:
        lx, ly, lz = self.edges[chain]
        out = np.empty((lz, ly, lx), dtype=np.float32)
        self._call(self.lib.batch_get_field, int(chain), _ptr(out))
        return out
