"""Host-only checks of the C-ABI library: it loads, exports every function
include/lbm.h declares, and rejects invalid arguments before touching a GPU.
No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lbm():
    from paper_0811_4593_amd import lbm as m
    m.load_library()
    return m


def test_header_declares_the_binding_exports(lbm):
    assert _declared_functions() == sorted(lbm.EXPORTS)


def test_library_exports_every_declared_symbol(lbm):
    lib = ctypes.CDLL(lbm.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_element_bytes(lbm):
    assert lbm.lbm_element_bytes(lbm.LBM_STORE_F64) == 8
    assert lbm.lbm_element_bytes(lbm.LBM_STORE_F32) == 4
    assert lbm.lbm_element_bytes(lbm.LBM_STORE_F16_DEV) == 2
    assert lbm.lbm_element_bytes(7) == 0


@pytest.mark.parametrize("args,frag", [
    ((0, 4, 4, 0.8), "sizes"),
    ((4, 4, 4, 0.5), "tau"),
    ((4, 4, 4, 0.4), "tau"),
    ((2048, 2048, 1024, 0.8), "2^31"),
])
def test_create_rejects_bad_arguments(lbm, args, frag):
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_create(*args)
    assert e.value.status == lbm.LBM_ERR_ARG
    assert frag in str(e.value)


def test_create_rejects_bad_storage_and_density(lbm):
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_create(4, 4, 4, 0.8, 1.0, None, 9)
    assert e.value.status == lbm.LBM_ERR_ARG
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_create(4, 4, 4, 0.8, -1.0)
    assert e.value.status == lbm.LBM_ERR_ARG


def test_create_on_buffers_validates(lbm):
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_create_on_buffers(4, 4, 4, 0.8, 1.0, None, lbm.LBM_STORE_F32, None, 0, 0, 0)
    assert e.value.status == lbm.LBM_ERR_ARG
    with pytest.raises(lbm.LBMError) as e:  # too small
        lbm.lbm_create_on_buffers(4, 4, 4, 0.8, 1.0, None, lbm.LBM_STORE_F32, None, 256, 512, 100)
    assert "needed" in str(e.value)
    with pytest.raises(lbm.LBMError) as e:  # misaligned
        lbm.lbm_create_on_buffers(4, 4, 4, 0.8, 1.0, None, lbm.LBM_STORE_F32, None, 4096 + 8, 8192, 1 << 20)
    assert "aligned" in str(e.value)


def test_null_handle_calls_fail_cleanly(lbm):
    lib = lbm.load_library()
    v = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    assert lib.lbm_set_velocity_bc(None, 0, v) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_pressure_bc(None, 4, 1.0, v) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_body_force(None, v) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_velocity_field(None, 4, v) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_solid_mask(None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_rule_options(None, 0) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_geometry(None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_autotune(None, 2, None, None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_get_step(None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_tune_placement(None, 4, 1, None, None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_classify_geometry(4, 4, 4, None, None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_step(None, 1) == lbm.LBM_ERR_ARG
    assert lib.lbm_clear_bc(None, 0) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_launch(None, 256, 1, 1) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_layout(None, lbm.LBM_LAYOUT_ROW_MAJOR) == lbm.LBM_ERR_ARG
    assert lib.lbm_batch_set_policy(None, lbm.LBM_BATCH_SHORTEST_FIRST, 0) == lbm.LBM_ERR_ARG
    assert lib.lbm_get_layout(None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_probe(None, 0, 1) == lbm.LBM_ERR_ARG
    assert lib.lbm_totals(None, None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_moments(None, None, None, 0) == lbm.LBM_ERR_ARG
    assert "NULL" in lbm.lbm_last_error()
    lib.lbm_destroy(None)  # no-op


def test_binding_refuses_to_run_without_library(tmp_path):
    from paper_0811_4593_amd import lbm as m
    saved = m._lib
    m._lib = None
    try:
        with pytest.raises(FileNotFoundError):
            m.load_library(str(tmp_path / "missing.so"))
    finally:
        m._lib = saved


def test_buffer_elements(lbm):
    F64, F32, F16 = lbm.LBM_STORE_F64, lbm.LBM_STORE_F32, lbm.LBM_STORE_F16_DEV
    POP, ROWS = lbm.LBM_LAYOUT_POPULATION_MAJOR, lbm.LBM_LAYOUT_ROW_MAJOR
    assert lbm.lbm_buffer_elements(37, 21, 13, F32, POP) == 19 * lbm.lbm_population_pitch(37 * 21 * 13)
    # row-major rows padded to 128 bytes: 32 FP32, 16 FP64, 64 FP16 elements
    assert lbm.lbm_buffer_elements(37, 21, 13, F32, ROWS) == 19 * 64 * 21 * 13
    assert lbm.lbm_buffer_elements(37, 21, 13, F64, ROWS) == 19 * 48 * 21 * 13
    assert lbm.lbm_buffer_elements(37, 21, 13, F16, ROWS) == 19 * 64 * 21 * 13
    assert lbm.lbm_buffer_elements(1024, 512, 512, F32, ROWS) == 19 * 1024 * 512 * 512
    assert lbm.lbm_buffer_elements(512, 256, 256, F16, ROWS) == 19 * 512 * 256 * 256
    assert lbm.lbm_buffer_elements(0, 4, 4, F32, ROWS) == 0
    assert lbm.lbm_buffer_elements(4, 4, 4, 9, ROWS) == 0
    assert lbm.lbm_buffer_elements(4, 4, 4, F32, 2) == 0


def test_population_pitch(lbm):
    assert lbm.lbm_population_pitch(64) == 64
    assert lbm.lbm_population_pitch(65) == 128
    assert lbm.lbm_population_pitch(1) == 64
    assert lbm.lbm_population_pitch(1024 * 512 * 512) == 1024 * 512 * 512
    assert lbm.lbm_population_pitch(221 * 17 * 93) % 64 == 0


def test_binding_checks_node_types_before_converting(lbm):
    """A node-type array is checked before it is cast to bytes: values that a
    cast would wrap (256 -> 0) or truncate (0.5 -> 0) are refused, and so is
    an array of the wrong size."""
    import numpy as np
    ok = np.zeros((3, 4, 5), np.int64)
    ok[0, 0, 0] = 2
    ok[1, 1, 1] = 1
    code, counts = lbm.lbm_classify_geometry(ok)
    assert code.shape == (3, 4, 5) and sum(counts) == 60
    for bad in (np.full((3, 4, 5), 256), np.full((3, 4, 5), 0.5), np.full((3, 4, 5), -1)):
        with pytest.raises(ValueError):
            lbm.lbm_classify_geometry(bad)
    with pytest.raises(ValueError):
        lbm._node_types(np.zeros(59, np.uint8), 60, "geometry")


def test_binding_checks_host_array_sizes(lbm):
    import numpy as np
    a = lbm._host_array(np.zeros(12), np.float64, 12, "x")
    assert a.size == 12
    with pytest.raises(ValueError):
        lbm._host_array(np.zeros(11), np.float64, 12, "x")
    with pytest.raises(ValueError):  # an output array must be writable float64 of the exact size
        lbm._host_array(np.zeros(12, np.float32), np.float64, 12, "x", writable=True)
    out = np.zeros(12)
    assert lbm._host_array(out, np.float64, 12, "x", writable=True) is out


def test_null_handle_calls_of_the_newer_entry_points(lbm):
    lib = lbm.load_library()
    assert lib.lbm_get_size(None, None, None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_set_steps_per_pass(None, 2, 0, 0) == lbm.LBM_ERR_ARG
    assert lib.lbm_get_steps_per_pass(None, None, None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_batch_set_lanes(None, 2) == lbm.LBM_ERR_ARG
    assert lib.lbm_batch_get_stats(None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_totals_static(None, 4, 4, 4, 1, 0, None, None) == lbm.LBM_ERR_ARG
    assert lib.lbm_batch_set_steps_per_pass(None, 2, 0) == lbm.LBM_ERR_ARG
    assert lib.lbm_batch_get_steps_per_pass(None, None, None) == lbm.LBM_ERR_ARG


@pytest.mark.parametrize("nx,ny,nz,storage", [(37, 12, 9, "f32"), (32, 10, 7, "f32"), (70, 9, 5, "f16dev"),
                                              (21, 11, 13, "f64"), (1, 1, 1, "f32")])
def test_job_bytes_cover_either_batch_layout(lbm, nx, ny, nz, storage):
    """A batch stores a job row-major with padded rows (two steps per pass)
    or, with one step per pass, population-major where its rows are not whole
    128-byte lines: lbm_job_bytes is the larger of the two."""
    from paper_0811_4593_amd import serving, workloads
    st = serving.STORAGE[storage]
    esize = lbm.lbm_element_bytes(st)

    def need(layout):
        buf = lbm.lbm_buffer_elements(nx, ny, nz, st, layout) * esize
        return 2 * ((buf + 255) // 256 * 256) + (3 * nx * ny * nz * 4 + 255) // 256 * 256

    spec = workloads.LatticeSpec(nx, ny, nz, 0.8, {}, name="box")
    got = lbm.lbm_job_bytes(serving.job_for(spec, storage, 0.0, 10))
    assert got == max(need(lbm.LBM_LAYOUT_ROW_MAJOR), need(lbm.LBM_LAYOUT_POPULATION_MAJOR))
