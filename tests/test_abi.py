"""The C ABI on the host (no GPU): libdem.so loads and exports every function
include/dem.h declares, and its host-only calls (status text, last error,
admission footprint) behave as documented."""
import ctypes as C
import os

import pytest

from paper_1607_02427_amd import dem, inputs as I

HAVE_LIB = os.path.exists(dem.LIB_PATH)
pytestmark = pytest.mark.skipif(not HAVE_LIB, reason="libdem.so is not built")


def test_header_declares_the_documented_entry_points():
    names = dem.declared_functions()
    for n in ("dem_create_system", "dem_destroy_system", "dem_build_celllist", "dem_compute_forces", "dem_step",
              "dem_energy", "dem_get_outputs", "dem_get_state", "dem_set_state", "dem_batch_create", "dem_batch_add",
              "dem_batch_remove", "dem_batch_step", "dem_footprint_bytes", "dem_status_string", "dem_last_error"):
        assert n in names, n


def test_library_exports_every_declared_function():
    L = dem.lib()
    missing = [n for n in dem.declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    L = dem.lib()
    texts = [L.dem_status_string(k).decode() for k in range(8)]
    assert all(texts) and len(set(texts)) == 8
    assert L.dem_status_string(99)  # unknown codes still give text
    assert L.dem_last_error(None) is not None


def test_footprint_grows_with_system_and_capacity():
    L = dem.lib()
    small = I.cubes_3d(n_side=8)
    large = I.cubes_3d(n_side=12)
    f_small = dem.footprint_bytes(small, "fp32")
    f_large = dem.footprint_bytes(large, "fp32")
    assert 0 < f_small < f_large
    # more row capacity, more bytes; FP64 records are larger than FP32 ones
    assert dem.footprint_bytes(small, "fp32", nbr_capacity=64) > dem.footprint_bytes(small, "fp32", nbr_capacity=32)
    assert dem.footprint_bytes(small, "fp64") > f_small
    p, keep = dem.make_params(small, "fp32")
    assert L.dem_footprint_bytes(C.byref(p)) == f_small
