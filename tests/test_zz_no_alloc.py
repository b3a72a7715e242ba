"""The entry point that allocates nothing (lbm_totals_static) against
lbm_totals, through the C ABI: the same FP64 mass and momentum, bit for bit,
on two calls in a row, the second on a smaller lattice (the static scratch
keeps the first call's partial sums and must not leak them into the
second)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0811_4593_amd import lbm, workloads  # noqa: E402


def _static_totals(h, storage, stream):
    lib = lbm.load_library()
    nx, ny, nz = lbm.lbm_get_size(h)
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    st = lib.lbm_totals_static(ctypes.c_void_p(lbm.lbm_state_buffer(h)), nx, ny, nz, storage,
                               lbm.lbm_get_layout(h), ctypes.c_void_p(stream.cuda_stream),
                               ctypes.c_void_p(out.data_ptr()))
    assert st == lbm.LBM_OK, lbm.lbm_last_error()
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("storage", [lbm.LBM_STORE_F64, lbm.LBM_STORE_F32, lbm.LBM_STORE_F16_DEV_SR])
def test_static_totals_equal_lbm_totals_on_two_calls(storage):
    stream = torch.cuda.current_stream()
    for spec, steps in ((workloads.duct(96, 40, 33, (0.04, 0.01, 0.01), 0.8), 7),
                        (workloads.duct(13, 7, 6, (0.02, 0.0, 0.01), 1.1), 3)):
        h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, storage, stream)
        try:
            for face, v in spec.bc.items():
                lbm.lbm_set_velocity_bc(h, face, v)
            lbm.lbm_step(h, steps)
            mass, mom = lbm.lbm_totals(h)
            got = _static_totals(h, storage, stream)
            print(f"{spec.name} storage {storage}: lbm_totals {mass!r}, static {got[0]!r}", flush=True)
            np.testing.assert_array_equal(got, np.array([mass, *mom]))
        finally:
            lbm.lbm_destroy(h)


def test_static_totals_population_major_and_errors():
    stream = torch.cuda.current_stream()
    spec = workloads.duct(37, 11, 9, (0.03, 0.01, 0.0), 0.9)
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, lbm.LBM_STORE_F32, stream)
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        lbm.lbm_set_layout(h, lbm.LBM_LAYOUT_POPULATION_MAJOR)
        lbm.lbm_step(h, 4)
        mass, mom = lbm.lbm_totals(h)
        np.testing.assert_array_equal(_static_totals(h, lbm.LBM_STORE_F32, stream), np.array([mass, *mom]))
        lib = lbm.load_library()
        buf = ctypes.c_void_p(lbm.lbm_state_buffer(h))
        out = torch.zeros(4, dtype=torch.float64, device="cuda")
        dst = ctypes.c_void_p(out.data_ptr())
        s = ctypes.c_void_p(stream.cuda_stream)
        assert lib.lbm_totals_static(None, 4, 4, 4, 1, 0, s, dst) == lbm.LBM_ERR_ARG
        assert lib.lbm_totals_static(buf, 4, 4, 4, 1, 0, s, None) == lbm.LBM_ERR_ARG
        assert lib.lbm_totals_static(buf, 0, 4, 4, 1, 0, s, dst) == lbm.LBM_ERR_ARG
        assert lib.lbm_totals_static(buf, 2048, 1024, 1024, 1, 0, s, dst) == lbm.LBM_ERR_ARG  # 2^31 nodes
        assert lib.lbm_totals_static(buf, 4, 4, 4, 9, 0, s, dst) == lbm.LBM_ERR_ARG
        assert lib.lbm_totals_static(buf, 4, 4, 4, 1, 5, s, dst) == lbm.LBM_ERR_ARG
    finally:
        lbm.lbm_destroy(h)
