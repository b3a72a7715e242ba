"""lbm_step(n) against n calls of lbm_step(1): bit-identical results, also when
the configuration changes between calls (moving walls, launch shape,
geometry options, the parity of the buffer holding the state)."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0811_4593_amd import lbm, workloads  # noqa: E402


def say(msg):
    print(msg, flush=True)


def _pair(spec, storage, solid=None):
    hs = []
    for _ in range(2):
        h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, 1.0, None, storage, torch.cuda.current_stream())
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        if solid is not None:
            lbm.lbm_set_solid_mask(h, solid)
        hs.append(h)
    return hs


def _state(h, spec):
    f = np.empty((19, spec.nz, spec.ny, spec.nx))
    return lbm.lbm_get_populations(h, f)


def _one_by_one(h, n):
    for _ in range(n):
        lbm.lbm_step(h, 1)


@pytest.mark.parametrize("storage", [lbm.LBM_STORE_F64, lbm.LBM_STORE_F32, lbm.LBM_STORE_F16_DEV,
                                     lbm.LBM_STORE_F16_DEV_SR])
def test_long_runs_equal_single_steps(storage):
    spec = workloads.couette(16, 16, 32, 0.05, 1.0)
    a, b = _pair(spec, storage)
    try:
        lbm.lbm_step(a, 77)
        _one_by_one(b, 77)
        np.testing.assert_array_equal(_state(a, spec), _state(b, spec))
        # moving wall
        for h in (a, b):
            lbm.lbm_set_velocity_bc(h, 5, (0.03, 0.01, 0.0))
        lbm.lbm_step(a, 64)
        _one_by_one(b, 64)
        np.testing.assert_array_equal(_state(a, spec), _state(b, spec))
        # other launch shape, odd parity on entry (the state is in the other buffer)
        for h in (a, b):
            lbm.lbm_set_launch(h, 128, 1, 0)
        lbm.lbm_step(a, 33)
        _one_by_one(b, 33)
        lbm.lbm_step(a, 96)
        _one_by_one(b, 96)
        np.testing.assert_array_equal(_state(a, spec), _state(b, spec))
    finally:
        for h in (a, b):
            lbm.lbm_destroy(h)


def test_long_runs_with_solid_mask_and_rule_option():
    st = workloads.tilted_channel(ny=2)
    s = st.spec
    a, b = _pair(s, lbm.LBM_STORE_F64, st.solid)
    try:
        for h in (a, b):
            for face, fv in st.face_v.items():
                lbm.lbm_set_velocity_field(h, face, fv)
        lbm.lbm_step(a, 70)
        _one_by_one(b, 70)
        np.testing.assert_array_equal(_state(a, s), _state(b, s))
        for h in (a, b):
            lbm.lbm_set_rule_options(h, lbm.LBM_RULE_NO_TRANSVERSE)
        lbm.lbm_step(a, 64)
        _one_by_one(b, 64)
        np.testing.assert_array_equal(_state(a, s), _state(b, s))
    finally:
        for h in (a, b):
            lbm.lbm_destroy(h)


def test_long_run_timing_small_lattice():
    spec = workloads.couette(16, 16, 32, 0.05, 1.0)
    a, b = _pair(spec, lbm.LBM_STORE_F64)
    try:
        lbm.lbm_step(a, 64)
        _one_by_one(b, 64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lbm.lbm_step(a, 3200)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        t0 = time.perf_counter()
        _one_by_one(b, 3200)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        say(f"16x16x32 FP64, 3200 steps: one call {tg * 1e3:.1f} ms, one call per step {tp * 1e3:.1f} ms")
        np.testing.assert_array_equal(_state(a, spec), _state(b, spec))
    finally:
        for h in (a, b):
            lbm.lbm_destroy(h)


def test_autotune_advances_real_steps_and_keeps_results():
    spec = workloads.duct(300, 20, 18, (0.04, 0.01, 0.01), 0.8)
    for storage in (lbm.LBM_STORE_F32, lbm.LBM_STORE_F16_DEV_SR):
        a, b = _pair(spec, storage)
        try:
            shape = lbm.lbm_autotune(a, 2)
            done = lbm.lbm_get_step(a)
            assert shape[0] in (64, 128, 256, 512) and shape[1] in (1, 2, 4) and done > 0
            assert lbm.lbm_get_launch(a) == shape
            lbm.lbm_step(a, 50)
            lbm.lbm_step(b, done + 50)
            assert lbm.lbm_get_step(a) == lbm.lbm_get_step(b) == done + 50
            np.testing.assert_array_equal(_state(a, spec), _state(b, spec))
            say(f"storage {storage}: autotuned {shape} in {done} steps")
        finally:
            for h in (a, b):
                lbm.lbm_destroy(h)
    h = lbm.lbm_create(8, 8, 8, 0.8, 1.0, None, lbm.LBM_STORE_F64, torch.cuda.current_stream())
    try:
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_autotune(h, 0)
        assert e.value.status == lbm.LBM_ERR_ARG
        lbm.lbm_set_velocity_bc(h, 4, (0.0, 0.0, 0.0))  # one face of an axis only
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_autotune(h, 2)
        assert e.value.status == lbm.LBM_ERR_STATE
    finally:
        lbm.lbm_destroy(h)


def test_tune_placement_keeps_the_state_and_counts_its_steps():
    """lbm_tune_placement moves the state between buffers and times real steps:
    afterwards the lattice equals one stepped plainly by the same count (FP32,
    and the stochastic-rounding form whose random words follow the step
    count), its state lies in one of the pool's buffers, and a lattice on
    caller-owned buffers is refused."""
    spec = workloads.duct(96, 20, 18, (0.04, 0.01, 0.01), 0.8)
    for storage, pool, trial in ((lbm.LBM_STORE_F32, 5, 1), (lbm.LBM_STORE_F16_DEV_SR, 3, 2)):
        a, b = _pair(spec, storage)
        try:
            lbm.lbm_step(a, 3)  # the state starts in the second buffer
            lbm.lbm_step(b, 3)
            before = lbm.lbm_state_buffer(a)
            tried, ms0, ms1 = lbm.lbm_tune_placement(a, pool, trial)
            pairs = tried * (tried - 1) // 2
            assert tried == pool and 0.0 < ms1 <= ms0
            assert lbm.lbm_get_step(a) == 3 + pairs * (2 + 2 * trial)
            lbm.lbm_step(a, 7)
            lbm.lbm_step(b, pairs * (2 + 2 * trial) + 7)
            np.testing.assert_array_equal(_state(a, spec), _state(b, spec))
            say(f"storage {storage}: {tried} buffers, {ms0:.4f} -> {ms1:.4f} ms/step, state moved: "
                f"{lbm.lbm_state_buffer(a) != before}")
        finally:
            for h in (a, b):
                lbm.lbm_destroy(h)
    h = lbm.lbm_create(8, 8, 8, 0.8, 1.0, None, lbm.LBM_STORE_F64, torch.cuda.current_stream())
    try:
        for bad in ((1, 1), (9, 1), (4, 0)):
            with pytest.raises(lbm.LBMError) as e:
                lbm.lbm_tune_placement(h, *bad)
            assert e.value.status == lbm.LBM_ERR_ARG
        tried, _, _ = lbm.lbm_tune_placement(h, 2, 1)  # the lattice's own pair only
        assert tried == 2 and lbm.lbm_get_step(h) == 4
    finally:
        lbm.lbm_destroy(h)
    P = lbm.lbm_population_pitch(8 * 8 * 8)
    bufs = [torch.empty(19 * P, dtype=torch.float64, device="cuda") for _ in range(2)]
    h = lbm.lbm_create_on_buffers(8, 8, 8, 0.8, 1.0, None, lbm.LBM_STORE_F64, torch.cuda.current_stream(),
                                  bufs[0], bufs[1], bufs[0].numel() * 8)
    try:
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_tune_placement(h, 4, 1)
        assert e.value.status == lbm.LBM_ERR_STATE
    finally:
        lbm.lbm_destroy(h)
