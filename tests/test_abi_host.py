"""Host-side checks of the C ABI (no GPU needed): the shared library loads and
exports every function include/polar.h declares, argument validation returns
the documented status codes before touching a device, the library's own
frozen-set construction agrees with the oracle's, and the BP kernel's
compile-time data layout passes the host verifier."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_1609_09358_amd import binding as PB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "polar.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    names = _declared()
    assert "hybrid_decode_batch" in names and "polar_build_code" in names and len(names) >= 12
    lib = C.CDLL(PB.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(PB.EXPORTED) == set(names)


def test_build_code_rejects_bad_arguments():
    lib = PB.lib()
    bad = [(100, 50, 0), (8192, 100, 0), (4, 2, 0), (128, 64, 12), (128, 0, 0), (128, 120, 16)]
    for N, K, c in bad:
        d = PB.polar_code_desc(N, K, c, 0, 2.0, None)
        h = C.c_void_p()
        assert lib.polar_build_code(C.byref(d), C.byref(h)) == 1, (N, K, c)
        assert not h.value
        assert lib.polar_last_error()
    # a given mask must freeze exactly N - K - c positions
    mask = np.ones(16, np.uint8)
    mask[:5] = 0
    d = PB.polar_code_desc(16, 4, 0, 0, 2.0, mask.ctypes.data_as(C.POINTER(C.c_uint8)))
    h = C.c_void_p()
    assert lib.polar_build_code(C.byref(d), C.byref(h)) == 1
    # CRC polynomial wider than the CRC
    d = PB.polar_code_desc(128, 64, 8, 0x1FF, 2.0, None)
    assert lib.polar_build_code(C.byref(d), C.byref(h)) == 1


def test_decoders_reject_null_code_without_device_work():
    lib = PB.lib()
    p = PB.make_bp_params()
    assert lib.bp_decode_batch(None, None, 0, C.byref(p), None, None, None, None, None) == 1
    assert lib.scl_decode_batch(None, None, 0, 8, None, None, None, None, None, 0, None) == 1
    assert lib.hybrid_decode_batch(None, None, 0, C.byref(p), 8, None, None, None, None, 0, None) == 1
    s = C.c_size_t()
    assert lib.polar_workspace_size(None, 1, 8, None, C.byref(s)) == 1
    assert lib.polar_encode(None, None, 0, None, None, None) == 1
    assert lib.hybrid_decode_pipelined(None, 1, None, 1, C.byref(p), 8, None, None, None, None, 0, None, None) == 1
    assert lib.polar_pipeline_workspace_size(None, 1, 8, C.byref(p), C.byref(s)) == 1
    h = C.c_void_p()
    assert lib.polar_mixed_create(None, 1, 16, C.byref(p), 8, None, C.byref(h)) == 1
    assert lib.polar_mixed_decode(None, 0, None, None, None, None, None, None, None, None) == 1
    assert lib.polar_mixed_decode_graph(None, 0, None, None, None, None, None, None, None, None) == 1
    lib.polar_mixed_free(None)


def test_scl_lds_budget_setter():
    lib = PB.lib()
    assert PB.polar_get_scl_lds_budget() == 0
    assert lib.polar_set_scl_lds_budget(100) == 1
    assert lib.polar_set_scl_lds_budget(200 * 1024) == 1
    assert PB.polar_get_scl_lds_budget() == 0
    PB.polar_set_scl_lds_budget(12288)
    assert PB.polar_get_scl_lds_budget() == 12288
    PB.polar_set_scl_lds_budget(0)
    assert PB.polar_get_scl_lds_budget() == 0


def test_pipeline_bp_occupancy_setter():
    lib = PB.lib()
    assert PB.polar_get_pipeline_bp_occupancy() == 0
    assert lib.polar_set_pipeline_bp_occupancy(-1) == 1
    assert lib.polar_set_pipeline_bp_occupancy(65) == 1
    PB.polar_set_pipeline_bp_occupancy(6)
    assert PB.polar_get_pipeline_bp_occupancy() == 6
    PB.polar_set_pipeline_bp_occupancy(0)
    assert PB.polar_get_pipeline_bp_occupancy() == 0


def test_pipeline_scl_occupancy_setter():
    lib = PB.lib()
    assert PB.polar_get_pipeline_scl_occupancy() == 0
    assert lib.polar_set_pipeline_scl_occupancy(-1) == 1
    assert lib.polar_set_pipeline_scl_occupancy(65) == 1
    PB.polar_set_pipeline_scl_occupancy(4)
    assert PB.polar_get_pipeline_scl_occupancy() == 4
    PB.polar_set_pipeline_scl_occupancy(0)
    assert PB.polar_get_pipeline_scl_occupancy() == 0


def test_scl_ranking_setter():
    lib = PB.lib()
    assert PB.polar_get_scl_ranking() == 0
    assert lib.polar_set_scl_ranking(4) == 1
    assert lib.polar_set_scl_ranking(-1) == 1
    for mode in (1, 2, 3):
        PB.polar_set_scl_ranking(mode)
        assert PB.polar_get_scl_ranking() == mode
    PB.polar_set_scl_ranking(0)


def test_bp_variants_query():
    assert PB.polar_bp_variants(1024) == [2, 3]
    assert PB.polar_bp_variants(8) == [2, 3]
    with pytest.raises(PB.PolarError):
        PB.polar_bp_variants(1000)


# (N, K, crc bits, design Eb/N0) of every code the workloads build
CODES = [(8, 4, 0, 2.0), (128, 64, 0, 2.0), (1024, 512, 16, 2.5), (256, 128, 8, 2.5), (1024, 512, 24, 2.5)] + [
    (N, int(N * R), 16, 2.0) for N in (256, 512, 1024, 2048) for R in (0.25, 0.5, 0.75)]


@pytest.mark.parametrize("N,K,c,e", CODES)
def test_library_construction_matches_oracle(N, K, c, e):
    lib_mask = PB.polar_construct_frozen(N, K, c, e)
    orc_mask = O.ga_frozen(N, K + c, e, K / N)
    assert np.array_equal(lib_mask, orc_mask)
    assert int((lib_mask == 0).sum()) == K + c


def test_bp_layout_verifier():
    exe = os.path.join(ROOT, "_build", "bp_geom_check")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    subprocess.check_call(["g++", "-std=c++20", "-O1", os.path.join(ROOT, "tests", "native", "bp_geom_check.cpp"),
                           "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout[-2000:]
    assert "all layouts verified" in out.stdout
