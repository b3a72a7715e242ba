"""Complex geometry on the GPU (Sec. V): wall nodes classified on the host,
rules in the extended sweep -- per-step FP64 parity against the oracle on a
ribbed channel and on random blocks, the box as a geometry against the
coordinate box, and FP32 against FP64 for the steady flow over a rib."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_0811_4593_amd import lbm, workloads  # noqa: E402
from test_oracle_complex_geometry import _box_geometry, _random_blocks  # noqa: E402


def say(msg):
    print(msg, flush=True)


def _gpu(nx, ny, nz, tau, storage, cell, force=None):
    h = lbm.lbm_create(nx, ny, nz, tau, 1.0, None, storage, torch.cuda.current_stream())
    assert cell.shape == (nz, ny, nx)
    lbm.lbm_set_geometry(h, cell)
    if force is not None:
        lbm.lbm_set_body_force(h, force)
    return h


def _cases():
    spec, cell = workloads.rib_channel()
    yield "rib", spec.tau, cell, (1e-5, 0.0, 0.0)
    for seed in (13, 18):
        yield f"blocks{seed}", 0.9, _random_blocks(seed), (0.0, 2e-6, -1e-6)
    yield "box", 0.8, _box_geometry(7, 6, 5), None


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_geometry_per_step_parity_fp64(case):
    name, tau, cell, force = case
    nz, ny, nx = cell.shape
    L = oracle.Lattice(nx, ny, nz, tau, cell=cell, force=force or (0.0, 0.0, 0.0))
    h = _gpu(nx, ny, nz, tau, lbm.LBM_STORE_F64, cell, force)
    try:
        lbm.lbm_set_populations(h, L.init(1.0, (0.01, 0.0, 0.005)) * workloads.perturbation(L.shape, 9, 0.05))
        cur, nxt = np.empty(L.shape), np.empty(L.shape)
        worst = 0.0
        live = cell != workloads.CELL_SOLID
        for _ in range(12):
            lbm.lbm_get_populations(h, cur)
            expect = L.step(cur)
            lbm.lbm_step(h, 1)
            lbm.lbm_get_populations(h, nxt)
            worst = max(worst, float(np.max(np.abs(nxt[:, live] - expect[:, live]) / np.abs(expect[:, live]))))
            np.testing.assert_array_equal(nxt[:, ~live], cur[:, ~live])  # solid interior untouched
        _, counts = lbm.lbm_classify_geometry(cell)
        say(f"{name}: kinds {counts}, worst rel diff {worst:.2e}")
        assert worst <= 1e-12
    finally:
        lbm.lbm_destroy(h)


def test_box_geometry_equals_coordinate_box_on_gpu():
    a, b, c = 9, 7, 6
    cell = _box_geometry(a, b, c)
    hb = lbm.lbm_create(a, b, c, 0.8, 1.0, None, lbm.LBM_STORE_F64, torch.cuda.current_stream())
    hg = _gpu(a + 2, b + 2, c + 2, 0.8, lbm.LBM_STORE_F64, cell)
    try:
        for f in range(6):
            lbm.lbm_set_velocity_bc(hb, f, (0.0, 0.0, 0.0))
        rng = np.random.default_rng(2)
        fb = oracle.Lattice(a, b, c, 0.8).init(1.0, (0.02, 0.01, -0.01)) * (1 + 0.05 * rng.uniform(-1, 1, (19, c, b, a)))
        fg = np.empty((19, c + 2, b + 2, a + 2))
        lbm.lbm_get_populations(hg, fg)
        fg[:, 1:-1, 1:-1, 1:-1] = fb
        lbm.lbm_set_populations(hb, fb)
        lbm.lbm_set_populations(hg, fg)
        lbm.lbm_step(hb, 20)
        lbm.lbm_step(hg, 20)
        lbm.lbm_get_populations(hb, fb)
        lbm.lbm_get_populations(hg, fg)
        diff = float(np.max(np.abs(fg[:, 1:-1, 1:-1, 1:-1] - fb) / np.abs(fb)))
        say(f"box as geometry vs coordinate box after 20 steps: {diff:.1e}")
        assert diff <= 1e-14
    finally:
        lbm.lbm_destroy(hb)
        lbm.lbm_destroy(hg)


def test_rib_flow_fp32_against_fp64():
    spec, cell = workloads.rib_channel(nx=48, ny=10, nz=18, rib=(16, 23, 8))
    out = {}
    for st in (lbm.LBM_STORE_F64, lbm.LBM_STORE_F32):
        h = _gpu(spec.nx, spec.ny, spec.nz, spec.tau, st, cell, (2e-6, 0.0, 0.0))
        try:
            lbm.lbm_step(h, 8000)
            u = np.empty(3 * spec.nodes)
            lbm.lbm_moments(h, None, u)
            out[st] = u.reshape(3, spec.nz, spec.ny, spec.nx)
        finally:
            lbm.lbm_destroy(h)
    live = cell != workloads.CELL_SOLID
    u64, u32 = out[lbm.LBM_STORE_F64][:, live], out[lbm.LBM_STORE_F32][:, live]
    e = float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64))
    say(f"rib channel FP32 vs FP64 rel L2 {e:.2e}, max u {np.abs(u64).max():.3e}")
    assert e <= 1e-5


def test_geometry_abi_errors():
    h = lbm.lbm_create(8, 8, 8, 0.8, 1.0, None, lbm.LBM_STORE_F64, torch.cuda.current_stream())
    try:
        bad = np.zeros((8, 8, 8), np.uint8)
        bad[3, 3, 3] = 3
        with pytest.raises(ValueError):  # the binding checks the node types first
            lbm.lbm_set_geometry(h, bad)
        # and the library itself refuses them
        st = lbm.load_library().lbm_set_geometry(h, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
        assert st == lbm.LBM_ERR_ARG
        cell = _box_geometry(6, 6, 6)
        lbm.lbm_set_geometry(h, cell)
        lbm.lbm_set_velocity_bc(h, 0, (0.0, 0.0, 0.0))
        lbm.lbm_set_velocity_bc(h, 1, (0.0, 0.0, 0.0))
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_step(h, 1)
        assert e.value.status == lbm.LBM_ERR_STATE
        lbm.lbm_clear_bc(h, 0)
        lbm.lbm_clear_bc(h, 1)
        lbm.lbm_set_solid_mask(h, np.zeros((8, 8, 8), np.uint8))
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_step(h, 1)
        assert e.value.status == lbm.LBM_ERR_STATE
        lbm.lbm_set_solid_mask(h, None)
        lbm.lbm_step(h, 2)
        lbm.lbm_set_geometry(h, None)
        lbm.lbm_step(h, 2)
    finally:
        lbm.lbm_destroy(h)
