"""Row-major population layout (lbm_set_layout): the same sweep on a
different placement of the populations in HBM, so every result must equal the
population-major one bit for bit -- every storage form, launch shape, the
pressure and force variants and both extended-sweep paths (solid mask with
per-node face velocities, complex geometry) -- plus one direct FP64 parity
check against the oracle and the full-size duct compared in device memory."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_0811_4593_amd import lbm, workloads  # noqa: E402
from test_oracle_complex_geometry import _random_blocks  # noqa: E402

POP, ROWS = lbm.LBM_LAYOUT_POPULATION_MAJOR, lbm.LBM_LAYOUT_ROW_MAJOR
WALL = (0.0, 0.0, 0.0)
FORMS = [lbm.LBM_STORE_F64, lbm.LBM_STORE_F32, lbm.LBM_STORE_F16_DEV, lbm.LBM_STORE_F16_DEV_SR]


def say(msg):
    print(msg, flush=True)


def _start(spec, seed=3, amp=0.05):
    L = oracle.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, bc=spec.bc)
    return L.init(spec.rho0, (0.01, 0.0, 0.005)) * workloads.perturbation(L.shape, seed, amp)


def _run(spec, storage, layout, steps, f0=None, launch=None, setup=None, layout_after_start=False):
    """Create a lattice, apply setup(h), set the state, step; returns
    (populations, rho, u, (mass, momentum))."""
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, storage, torch.cuda.current_stream())
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        if setup:
            setup(h)
        if launch:
            lbm.lbm_set_launch(h, *launch)
        if not layout_after_start:
            lbm.lbm_set_layout(h, layout)
        if f0 is not None:
            lbm.lbm_set_populations(h, f0)
        if layout_after_start:
            lbm.lbm_set_layout(h, layout)
        assert lbm.lbm_get_layout(h) == layout
        lbm.lbm_step(h, steps)
        f = np.empty((19, spec.nz, spec.ny, spec.nx))
        lbm.lbm_get_populations(h, f)
        rho, u = np.empty(spec.nodes), np.empty(3 * spec.nodes)
        lbm.lbm_moments(h, rho, u)
        return f, rho, u, lbm.lbm_totals(h)
    finally:
        lbm.lbm_destroy(h)


def _same(a, b):
    fa, ra, ua, ta = a
    fb, rb, ub, tb = b
    np.testing.assert_array_equal(fa, fb)
    np.testing.assert_array_equal(ra, rb)
    np.testing.assert_array_equal(ua, ub)
    assert ta[0] == tb[0] and np.array_equal(np.asarray(ta[1]), np.asarray(tb[1]))


@pytest.mark.parametrize("storage", FORMS, ids=lambda s: lbm.STORAGE_NAMES[s])
def test_duct_every_storage_form_bitwise(storage):
    """A ragged duct (37 = 64-lane blocks with idle lanes; faces, edges and
    corners on all six sides), 9 steps from a perturbed moving state."""
    spec = workloads.duct(37, 21, 13, (0.04, 0.01, 0.01), 0.8)
    f0 = _start(spec)
    ref = _run(spec, storage, POP, 9, f0)
    _same(_run(spec, storage, ROWS, 9, f0), ref)
    # switching after the state is set moves it without changing a bit
    _same(_run(spec, storage, ROWS, 9, f0, layout_after_start=True), ref)


@pytest.mark.parametrize("launch", [(64, 1, 0), (64, 2, 2), (128, 1, 1), (256, 4, 0), (512, 1, 2)])
def test_row_major_every_launch_shape_bitwise(launch):
    """150-node rows: 1 to 3 blocks per row with ragged last blocks, every
    XCD placement; FP32 row-major against the default shape population-major."""
    spec = workloads.duct(150, 11, 9, (0.03, -0.01, 0.02), 0.7)
    f0 = _start(spec, seed=4)
    ref = _run(spec, lbm.LBM_STORE_F32, POP, 7, f0)
    _same(_run(spec, lbm.LBM_STORE_F32, ROWS, 7, f0, launch=launch), ref)


def test_pressure_and_force_bitwise():
    """Pressure inlet/outlet with no-slip y/z walls (FP64), and a body force
    on a channel periodic in x and y (FP32)."""
    spec = workloads.LatticeSpec(24, 10, 9, 0.9, {2: WALL, 3: WALL, 4: WALL, 5: WALL}, name="pressure_duct")

    def pressure(h):
        lbm.lbm_set_pressure_bc(h, 0, 1.01)
        lbm.lbm_set_pressure_bc(h, 1, 0.99)

    f0 = _start(spec, seed=5, amp=0.02)
    _same(_run(spec, lbm.LBM_STORE_F64, ROWS, 8, f0, setup=pressure),
          _run(spec, lbm.LBM_STORE_F64, POP, 8, f0, setup=pressure))
    spec = workloads.LatticeSpec(16, 12, 10, 1.0, {4: WALL, 5: WALL}, name="force_channel")

    def force(h):
        lbm.lbm_set_body_force(h, (1e-5, 2e-6, 0.0))

    f0 = _start(spec, seed=6, amp=0.02)
    _same(_run(spec, lbm.LBM_STORE_F32, ROWS, 8, f0, setup=force),
          _run(spec, lbm.LBM_STORE_F32, POP, 8, f0, setup=force))


def test_extended_sweep_solid_mask_and_face_fields_bitwise():
    """Solid nodes (mid-grid bounce-back reads the node's own opposite
    population) and per-node face velocities, FP64 and FP16 with stochastic
    rounding."""
    rng = np.random.default_rng(21)
    nx, ny, nz = 70, 9, 10
    solid = (rng.uniform(size=(nz, ny, nx)) < 0.12).astype(np.uint8)
    solid[:, :, 0] = solid[:, :, -1] = 0
    fv = {0: rng.uniform(-0.02, 0.03, (nz, ny, 3)), 1: rng.uniform(-0.02, 0.03, (nz, ny, 3)),
          3: rng.uniform(-0.01, 0.01, (nz, nx, 3))}
    spec = workloads.LatticeSpec(nx, ny, nz, 0.85, {0: WALL, 1: WALL, 2: WALL, 3: WALL}, name="obstacles_70x9x10")

    def setup(h):
        for face, v in fv.items():
            lbm.lbm_set_velocity_field(h, face, v)
        lbm.lbm_set_solid_mask(h, solid)

    f0 = _start(spec, seed=7, amp=0.03)
    for storage in (lbm.LBM_STORE_F64, lbm.LBM_STORE_F16_DEV_SR):
        _same(_run(spec, storage, ROWS, 10, f0, setup=setup), _run(spec, storage, POP, 10, f0, setup=setup))


def test_extended_sweep_complex_geometry_bitwise():
    """Complex geometry (node codes: plane, edge and corner walls, convex
    edges, general wall nodes, solid interiors) under a body force, FP64."""
    cell = _random_blocks(13)
    nz, ny, nx = cell.shape
    spec = workloads.LatticeSpec(nx, ny, nz, 0.9, {}, name="blocks13")

    def setup(h):
        lbm.lbm_set_geometry(h, cell)
        lbm.lbm_set_body_force(h, (0.0, 2e-6, -1e-6))

    _same(_run(spec, lbm.LBM_STORE_F64, ROWS, 12, None, setup=setup),
          _run(spec, lbm.LBM_STORE_F64, POP, 12, None, setup=setup))


def test_row_major_fp64_step_parity_with_oracle():
    """Row-major FP64 against the oracle directly, step by step (the same
    1e-12 bar as the population-major parity tests)."""
    spec = workloads.duct(21, 9, 8, (0.04, 0.01, 0.01), 0.8)
    L = oracle.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, bc=spec.bc)
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, lbm.LBM_STORE_F64,
                       torch.cuda.current_stream())
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        lbm.lbm_set_layout(h, ROWS)
        lbm.lbm_set_populations(h, L.init(1.0) * workloads.perturbation(L.shape, 9, 0.05))
        cur, nxt = np.empty(L.shape), np.empty(L.shape)
        worst = 0.0
        for _ in range(4):
            lbm.lbm_get_populations(h, cur)
            expect = L.step(cur)
            lbm.lbm_step(h, 1)
            lbm.lbm_get_populations(h, nxt)
            worst = max(worst, float(np.max(np.abs(nxt - expect) / np.abs(expect))))
        say(f"row-major fp64 vs oracle: max rel diff {worst:.2e}")
        assert worst <= 1e-12
    finally:
        lbm.lbm_destroy(h)


def test_layout_round_trip_and_errors():
    """A lattice of lbm_create starts row-major; rows -> pop -> rows restores
    the state bit for bit, each switch moving it to the pair's other buffer
    (the library's pair holds either layout); an unknown layout is rejected
    and changes nothing."""
    spec = workloads.duct(19, 7, 6)
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, 1.0, None, lbm.LBM_STORE_F16_DEV,
                       torch.cuda.current_stream())
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        assert lbm.lbm_get_layout(h) == ROWS
        lbm.lbm_step(h, 5)
        before = np.empty((19, spec.nz, spec.ny, spec.nx))
        lbm.lbm_get_populations(h, before)
        b0 = lbm.lbm_state_buffer(h)
        lbm.lbm_set_layout(h, ROWS)  # no-op
        assert lbm.lbm_state_buffer(h) == b0
        lbm.lbm_set_layout(h, POP)
        assert lbm.lbm_state_buffer(h) != b0 and lbm.lbm_get_layout(h) == POP
        mid = np.empty_like(before)
        lbm.lbm_get_populations(h, mid)
        np.testing.assert_array_equal(mid, before)
        lbm.lbm_set_layout(h, ROWS)
        assert lbm.lbm_state_buffer(h) == b0
        after = np.empty_like(before)
        lbm.lbm_get_populations(h, after)
        np.testing.assert_array_equal(after, before)
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_set_layout(h, 2)
        assert e.value.status == lbm.LBM_ERR_ARG
        assert lbm.lbm_get_layout(h) == ROWS
    finally:
        lbm.lbm_destroy(h)


def test_caller_owned_buffers_must_hold_the_padded_rows():
    """37-wide rows pad to 64 FP32 elements: caller buffers sized for the
    population-major layout are refused (layout unchanged), buffers of
    lbm_buffer_elements bytes work and give the same bits; a lattice on the
    library's buffers holds both layouts."""
    spec = workloads.duct(37, 9, 7)
    nx, ny, nz, N = spec.nx, spec.ny, spec.nz, spec.nodes
    stream = torch.cuda.current_stream()
    f0 = _start(spec, seed=12)
    ref = _run(spec, lbm.LBM_STORE_F32, POP, 6, f0)
    small = [torch.empty(19 * lbm.lbm_population_pitch(N), dtype=torch.float32, device="cuda") for _ in range(2)]
    need = lbm.lbm_buffer_elements(nx, ny, nz, lbm.LBM_STORE_F32, ROWS)
    assert need == 19 * 64 * ny * nz > small[0].numel()
    big = [torch.empty(need, dtype=torch.float32, device="cuda") for _ in range(2)]
    for bufs, ok in ((small, False), (big, True)):
        h = lbm.lbm_create_on_buffers(nx, ny, nz, spec.tau, 1.0, None, lbm.LBM_STORE_F32, stream,
                                      bufs[0], bufs[1], bufs[0].numel() * 4)
        try:
            for face, v in spec.bc.items():
                lbm.lbm_set_velocity_bc(h, face, v)
            lbm.lbm_set_populations(h, f0)
            if not ok:
                with pytest.raises(lbm.LBMError) as e:
                    lbm.lbm_set_layout(h, ROWS)
                assert e.value.status == lbm.LBM_ERR_STATE
                assert lbm.lbm_get_layout(h) == POP
                continue
            lbm.lbm_set_layout(h, ROWS)
            assert lbm.lbm_state_buffer(h) in (bufs[0].data_ptr(), bufs[1].data_ptr())
            lbm.lbm_step(h, 6)
            f = np.empty((19, nz, ny, nx))
            lbm.lbm_get_populations(h, f)
            np.testing.assert_array_equal(f, ref[0])
            # the device state as documented: element k R + 19 R r + x, R = 64
            cur = bufs[0] if lbm.lbm_state_buffer(h) == bufs[0].data_ptr() else bufs[1]
            dev = cur.view(nz, ny, 19, 64)[..., :nx].permute(2, 0, 1, 3).double().cpu().numpy()
            W = np.array([2] * 6 + [1] * 12 + [12]) / 36.0
            np.testing.assert_array_equal(dev + W[:, None, None, None], f)
        finally:
            lbm.lbm_destroy(h)
    h = lbm.lbm_create(nx, ny, nz, spec.tau, 1.0, None, lbm.LBM_STORE_F32, stream)
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        lbm.lbm_set_populations(h, f0)
        assert lbm.lbm_get_layout(h) == ROWS  # the library's pair holds the padded rows from the start
        lbm.lbm_set_layout(h, POP)
        lbm.lbm_set_layout(h, ROWS)
        lbm.lbm_step(h, 6)
        f = np.empty((19, nz, ny, nx))
        lbm.lbm_get_populations(h, f)
        np.testing.assert_array_equal(f, ref[0])
    finally:
        lbm.lbm_destroy(h)


@pytest.mark.slow
def test_full_size_duct_row_major_equals_population_major_in_device_memory():
    """The 1024x512x512 FP32 duct in the default launch shape: 3 steps in each
    layout on caller-owned buffers, then the two stored states compared
    element by element on the device (row-major viewed as [row][k][x])."""
    spec = workloads.roofline_duct()
    nx, ny, nz, N = spec.nx, spec.ny, spec.nz, spec.nodes
    P = lbm.lbm_population_pitch(N)
    assert lbm.lbm_buffer_elements(nx, ny, nz, lbm.LBM_STORE_F32, ROWS) == 19 * N  # 1024-wide rows: no padding
    say(f"full-size duct {nx}x{ny}x{nz} fp32, both layouts: allocating 4 x {19 * P * 4 / 1e9:.1f} GB")
    stream = torch.cuda.current_stream()
    states = {}
    for layout in (POP, ROWS):
        bufs = [torch.empty(19 * P, dtype=torch.float32, device="cuda") for _ in range(2)]
        h = lbm.lbm_create_on_buffers(nx, ny, nz, spec.tau, 1.0, None, lbm.LBM_STORE_F32, stream,
                                      bufs[0], bufs[1], bufs[0].numel() * 4)
        try:
            for face, v in spec.bc.items():
                lbm.lbm_set_velocity_bc(h, face, v)
            lbm.lbm_set_layout(h, layout)
            lbm.lbm_step(h, 3)
            torch.cuda.synchronize()
            cur = 0 if lbm.lbm_state_buffer(h) == bufs[0].data_ptr() else 1
            states[layout] = bufs[cur]
        finally:
            lbm.lbm_destroy(h)
        del bufs
    pop = states[POP].view(19, P)[:, :N]
    rows = states[ROWS][:19 * N].view(nz * ny, 19, nx).permute(1, 0, 2).reshape(19, N)
    equal = bool(torch.equal(pop, rows))
    say(f"  states equal: {equal}")
    assert equal
