"""MI355X-native heat-bath estimator of the lattice N-body Coulomb energy.

The N-body Coulomb energy E_N = sum_{i != j} q_i q_j G(n_i, n_j) is written
as an average over a free scalar field on a cubic lattice (the path-integral
representation of the lattice Green's function G = (-Delta_L)^{-1}) and
estimated by a red-black Gaussian heat bath run in hand-written HIP kernels.

The native library is loaded lazily: ``import paper_1403_0711_amd`` works
without it, and the first use of :class:`Lattice` or :class:`Batch` raises if
it has not been built.
"""

import importlib

__all__ = ["Lattice", "Batch", "LatticeError", "load_library"]


def __getattr__(name):
    if name in __all__:
        return getattr(importlib.import_module(__name__ + ".lattice"), name)
    raise AttributeError(name)
