"""Two steps per pass (lbm_set_steps_per_pass(h, 2)): the state after every
pair of steps equals, bit for bit, the state after two single sweeps, in all
four storage forms, on lattices whose extents are not multiples of the tile
(64 x 13 or 64 x 5 nodes) or of the z range, with every node class, moving
walls, pressure faces, a body force and the rule without N; and at full size
on the 1024 x 512 x 512 FP32 duct the bench times.  The single sweep is
parity-pinned to the oracle (test_gpu_parity.py), and one FP64 pair is also
checked against two oracle steps directly."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_0811_4593_amd import lbm, serving, workloads  # noqa: E402

STORAGES = [lbm.LBM_STORE_F64, lbm.LBM_STORE_F32, lbm.LBM_STORE_F16_DEV, lbm.LBM_STORE_F16_DEV_SR]


def say(msg):
    print(msg, flush=True)


INT_OF = {8: torch.int64, 4: torch.int32, 2: torch.int16}


def _lattice(spec, storage, force=None, no_n=False, state=None):
    """A lattice on two zero-filled caller-owned buffers (torch tensors of the
    element width as integers, so their bits can be compared), row-major."""
    esize = lbm.lbm_element_bytes(storage)
    n = max(lbm.lbm_buffer_elements(spec.nx, spec.ny, spec.nz, storage, lbm.LBM_LAYOUT_ROW_MAJOR),
            lbm.lbm_buffer_elements(spec.nx, spec.ny, spec.nz, storage, lbm.LBM_LAYOUT_POPULATION_MAJOR))
    bufs = [torch.zeros(n, dtype=INT_OF[esize], device="cuda") for _ in range(2)]
    h = lbm.lbm_create_on_buffers(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, storage,
                                  torch.cuda.current_stream(), bufs[0], bufs[1], n * esize)
    serving.apply_bc(h, spec)
    if force is not None:
        lbm.lbm_set_body_force(h, force)
    if no_n:
        lbm.lbm_set_rule_options(h, lbm.LBM_RULE_NO_TRANSVERSE)
    if state is not None:
        lbm.lbm_set_populations(h, state)
    lbm.lbm_set_layout(h, lbm.LBM_LAYOUT_ROW_MAJOR)
    return h, bufs


def _raw_state(h, bufs, spec, storage):
    """The stored encodings of the nodes (padding excluded), as integers."""
    torch.cuda.synchronize()
    cur = bufs[0] if lbm.lbm_state_buffer(h) == bufs[0].data_ptr() else bufs[1]
    assert lbm.lbm_state_buffer(h) == cur.data_ptr()
    R = lbm.lbm_buffer_elements(spec.nx, 1, 1, storage, lbm.LBM_LAYOUT_ROW_MAJOR) // 19
    return cur[:19 * R * spec.ny * spec.nz].view(spec.nz, spec.ny, 19, R)[..., :spec.nx]


CASES = [
    (workloads.duct(130, 27, 9, (0.04, 0.01, 0.01), 0.8), None, False),
    (workloads.duct(67, 14, 70, (0.03, -0.02, 0.015), 0.7), None, False),
    (workloads.all_classes_lattices()[2], None, False),
    (workloads.all_classes_lattices()[3], (1e-5, -2e-5, 3e-5), False),
    (workloads.all_classes_lattices()[4], None, True),
    (workloads.pressure_classes_lattices()[0], None, False),
    (workloads.pressure_classes_lattices()[1], (2e-5, 0.0, 1e-5), False),
    (workloads.LatticeSpec(5, 3, 4, 0.9, {}, name="periodic_5x3x4"), (1e-4, 0.0, 0.0), False),
]


@pytest.mark.parametrize("rows", [0, 5, 12], ids=["default-tiles", "5-row-tiles", "12-row-tiles"])
@pytest.mark.parametrize("storage", STORAGES, ids=lambda s: lbm.STORAGE_NAMES[s])
@pytest.mark.parametrize("case", range(len(CASES)), ids=lambda i: CASES[i][0].name)
def test_two_steps_per_pass_equal_two_single_sweeps(case, storage, rows):
    spec, force, no_n = CASES[case]
    f0 = oracle.Lattice(spec.nx, spec.ny, spec.nz, spec.tau).init(1.0, (0.01, 0.0, 0.005)) * \
        workloads.perturbation((19, spec.nz, spec.ny, spec.nx), 11, 0.05)
    a, abufs = _lattice(spec, storage, force, no_n, f0)
    b, bbufs = _lattice(spec, storage, force, no_n, f0)
    try:
        lbm.lbm_set_steps_per_pass(b, 2, 4 if spec.nz > 8 else 0, rows)
        for steps in (2, 4, 3):  # pairs, and an odd count (the last step single)
            lbm.lbm_step(a, steps)
            lbm.lbm_step(b, steps)
            assert lbm.lbm_get_step(a) == lbm.lbm_get_step(b)
            ra, rb = _raw_state(a, abufs, spec, storage), _raw_state(b, bbufs, spec, storage)
            assert torch.equal(ra, rb), f"{spec.name}: states differ after {lbm.lbm_get_step(a)} steps"
    finally:
        lbm.lbm_destroy(a)
        lbm.lbm_destroy(b)


def test_two_step_pass_fp64_against_oracle():
    spec = workloads.all_classes_lattices()[1]
    L = oracle.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, bc=spec.bc)
    f = L.init(1.0, (0.02, 0.0, 0.01)) * workloads.perturbation(L.shape, 3, 0.05)
    h, _ = _lattice(spec, lbm.LBM_STORE_F64, state=f)
    try:
        lbm.lbm_set_steps_per_pass(h, 2, 0)
        worst = 0.0
        got = np.empty(L.shape)
        for _ in range(5):
            lbm.lbm_get_populations(h, got)
            expect = L.step(L.step(got))
            lbm.lbm_step(h, 2)
            lbm.lbm_get_populations(h, got)
            worst = max(worst, float(np.max(np.abs(got - expect) / np.abs(expect))))
        say(f"two-step pass vs two oracle steps: worst rel diff {worst:.2e}")
        assert worst <= 2e-12
    finally:
        lbm.lbm_destroy(h)


@pytest.mark.parametrize("rows", [0, 5, 12], ids=["default-tiles", "5-row-tiles", "12-row-tiles"])
def test_two_step_pass_full_size_duct_equals_single_sweeps(rows):
    """The bench's workload and launch (1024 x 512 x 512 FP32 duct, row-major,
    default z ranges): after six steps from rest, every element of the state
    equals the single-sweep state."""
    spec = workloads.roofline_duct()
    a, abufs = _lattice(spec, lbm.LBM_STORE_F32)
    b, bbufs = _lattice(spec, lbm.LBM_STORE_F32)
    try:
        lbm.lbm_set_steps_per_pass(b, 2, 32, rows)
        lbm.lbm_step(a, 6)
        lbm.lbm_step(b, 6)
        ra, rb = _raw_state(a, abufs, spec, lbm.LBM_STORE_F32), _raw_state(b, bbufs, spec, lbm.LBM_STORE_F32)
        diff = int((ra != rb).sum())
        say(f"full-size duct, 6 steps: {diff} of {ra.numel()} elements differ")
        assert diff == 0
    finally:
        lbm.lbm_destroy(a)
        lbm.lbm_destroy(b)
        del abufs, bbufs
        torch.cuda.empty_cache()


def test_steps_per_pass_arguments():
    h = lbm.lbm_create(8, 8, 8, 0.8)
    try:
        assert lbm.lbm_get_steps_per_pass(h) == (1, 64, 0)
        for bad in ((0, 0, 0), (3, 0, 0), (2, -1, 0), (2, 0, 7), (2, 0, 9)):
            with pytest.raises(lbm.LBMError) as e:
                lbm.lbm_set_steps_per_pass(h, *bad)
            assert e.value.status == lbm.LBM_ERR_ARG
        lbm.lbm_set_steps_per_pass(h, 2, 16, 5)
        assert lbm.lbm_get_steps_per_pass(h) == (2, 16, 5)
        lbm.lbm_set_steps_per_pass(h, 2, 16, 12)
        assert lbm.lbm_get_steps_per_pass(h) == (2, 16, 12)
    finally:
        lbm.lbm_destroy(h)
