"""The C-ABI library loads and exports every symbol its header declares, and
argument validation that happens before any device work (CPU only)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lattice_coulomb.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*([a-z_]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1403_0711_amd import lattice

    if not os.path.exists(lattice.LIB_PATH):
        from paper_1403_0711_amd import build_lib

        build_lib.build()
    return lattice.load_library()


def test_header_declares_the_method_calls():
    names = _declared_functions()
    for n in ("lattice_create", "set_charges", "thermalise", "sweep_and_measure", "energy_estimate",
              "lattice_destroy", "lattice_last_error", "batch_create", "batch_run"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in _declared_functions():
        assert hasattr(lib, n), n


def test_create_validation_without_device(lib):
    """Invalid boxes are rejected before any HIP call."""
    h = ctypes.c_void_p()
    for args in ((3, 4, 4), (0, 4, 4), (4, 0, 4), (4, 4, -1), (2048, 1024, 1024)):
        rc = lib.lattice_create(*args, 0, 0, 0, None, None, ctypes.byref(h))
        assert rc == 1, args
        assert not h.value
    rc = lib.lattice_create(4, 4, 4, 7, 0, 0, None, None, ctypes.byref(h))
    assert rc == 1 and b"storage" in lib.lattice_last_error()
    assert lib.lattice_create(4, 4, 4, 0, 0, 0, None, None, None) == 1


def test_null_handles_are_rejected(lib):
    assert lib.thermalise(None, 1) == 1
    assert lib.sweep_and_measure(None, 1, 1, 1) == 1
    assert lib.energy_estimate(None, None, None, None, None) == 1
    assert lib.lattice_set_charge_sets(None, 1, None, None, None) == 1
    assert lib.lattice_energy_estimate_set(None, 0, None, None, None, None) == 1
    assert lib.lattice_get_sample_path(None, None) == 1
    lib.lattice_destroy(None)
