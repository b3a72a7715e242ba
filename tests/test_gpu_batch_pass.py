"""Two steps per pass in the batch runtime (lbm_batch_set_steps_per_pass):
in mode 2 one launch per storage form advances every job of a chunk by two
steps over the 64 x 13 (FP64: 64 x 5) tiles and z ranges of all its jobs; a
chunk of one job runs the single-lattice two-step kernel.  Bar: every job ends bitwise
equal to the same lattice advanced alone with lbm_step (single sweeps), for
chunk lengths that need only passes (a multiple of 4 steps) and ones that
close with two single steps, every storage form, lattices narrower or
shorter than one tile or one z range, and every scheduling policy."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0811_4593_amd import lbm, serving, workloads  # noqa: E402
from test_gpu_batch import MIX, _submit_all  # noqa: E402


def say(msg):
    print(msg, flush=True)


def _run_all(b):
    while lbm.lbm_batch_run_chunk(b) != (0, 0):
        pass


def _check_alone(b, ids, items, steps=None):
    """Every job done (after `steps` steps, if given) and bitwise equal to
    the lattice advanced alone by as many steps."""
    for jid, (spec, st) in zip(ids, items):
        s = lbm.lbm_batch_poll(b, jid)
        assert s.state == lbm.LBM_JOB_DONE and (steps is None or s.steps == steps), (spec.name, s.steps)
        rho_b, u_b = lbm.lbm_batch_result(b, jid, spec.nodes)
        _, rho_p, u_p = serving.run_plain(spec, st, s.steps)
        np.testing.assert_array_equal(rho_b, rho_p, err_msg=f"{spec.name} {st}")
        np.testing.assert_array_equal(u_b, u_p, err_msg=f"{spec.name} {st}")


def test_one_step_per_launch_is_the_default():
    b = lbm.lbm_batch_create(1 << 30, 10, 4)
    try:
        assert lbm.lbm_batch_get_steps_per_pass(b) == (1, 32)
    finally:
        lbm.lbm_batch_destroy(b)


@pytest.mark.parametrize("chunk,z_planes", [(12, 0), (10, 0), (8, 3), (4, 64), (2, 0)],
                         ids=["passes-only", "passes-and-2-single", "z3", "z64", "single-steps-only"])
def test_pass_batch_equals_alone_bitwise(chunk, z_planes):
    steps = 3 * chunk
    b = lbm.lbm_batch_create(4 << 30, chunk, 16)
    try:
        lbm.lbm_batch_set_steps_per_pass(b, 2, z_planes)
        ids = _submit_all(b, MIX, steps)
        _run_all(b)
        _check_alone(b, ids, MIX, steps)
    finally:
        lbm.lbm_batch_destroy(b)


def test_one_step_per_pass_equals_alone_bitwise():
    steps = 30
    b = lbm.lbm_batch_create(4 << 30, 10, 16)
    try:
        lbm.lbm_batch_set_steps_per_pass(b, 1, 0)
        ids = _submit_all(b, MIX, steps)
        _run_all(b)
        _check_alone(b, ids, MIX, steps)
    finally:
        lbm.lbm_batch_destroy(b)


@pytest.mark.parametrize("policy", [lbm.LBM_BATCH_SHORTEST_FIRST, lbm.LBM_BATCH_LARGE_IN_ORDER],
                         ids=["shortest-first", "large-in-order"])
def test_pass_solo_and_shared_chunks_equal_alone(policy):
    """Chunks of one job (the single-lattice two-step kernel) and chunks that
    share a launch, on three lanes."""
    items = MIX[:6]
    steps = 24
    b = lbm.lbm_batch_create(4 << 30, 12, 16)
    try:
        lbm.lbm_batch_set_steps_per_pass(b, 2, 0)
        lbm.lbm_batch_set_policy(b, policy, 2000)
        lbm.lbm_batch_set_lanes(b, 3)
        ids = _submit_all(b, items, steps)
        _run_all(b)
        stats = lbm.lbm_batch_get_stats(b)
        say(f"policy {policy}: {stats}")
        _check_alone(b, ids, items, steps)
    finally:
        lbm.lbm_batch_destroy(b)


def test_pass_autotune_keeps_results():
    items = MIX[:5]
    b = lbm.lbm_batch_create(4 << 30, 20, 8)
    try:
        lbm.lbm_batch_set_steps_per_pass(b, 2, 0)
        ids = _submit_all(b, items, 100)
        shape = lbm.lbm_batch_autotune(b, 4)
        sp, zc = lbm.lbm_batch_get_steps_per_pass(b)
        say(f"autotuned {shape}, pass {sp} z {zc}")
        assert sp == 2 and zc in (16, 32, 64)
        _run_all(b)
        _check_alone(b, ids, items)  # the trial steps are real steps: at least 100
    finally:
        lbm.lbm_batch_destroy(b)


def test_pass_mode_arguments_and_state():
    b = lbm.lbm_batch_create(1 << 30, 10, 4)
    try:
        for bad in ((0, 0), (3, 0), (2, -1), (2, 5000)):
            with pytest.raises(lbm.LBMError) as e:
                lbm.lbm_batch_set_steps_per_pass(b, *bad)
            assert e.value.status == lbm.LBM_ERR_ARG
        lbm.lbm_batch_set_steps_per_pass(b, 1, 16)
        # with one step per pass a job whose rows are not whole lines is stored
        # population-major, and the two-step mode is then refused
        spec = workloads.duct(37, 12, 9, (0.04, 0.01, 0.01), 0.8)
        jid = lbm.lbm_batch_submit(b, serving.job_for(spec, "f32", 0.0, 10))
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_batch_set_steps_per_pass(b, 2, 0)
        assert e.value.status == lbm.LBM_ERR_STATE
        assert lbm.lbm_batch_get_steps_per_pass(b) == (1, 16)
        _run_all(b)
        lbm.lbm_batch_result(b, jid, spec.nodes)
        lbm.lbm_batch_set_steps_per_pass(b, 2, 0)  # nothing queued or resident
        assert lbm.lbm_batch_get_steps_per_pass(b) == (2, 32)
    finally:
        lbm.lbm_batch_destroy(b)


def test_pass_batch_of_uneven_ducts_equals_plain():
    """Sixteen of the benchmark's uneven ducts (Nx ~ U{32..256}, Ny, Nz ~
    U{16..128}) in one batch, two steps per pass, against plain launches."""
    specs = workloads.batch_ducts(16, seed=3)
    run = serving.run_batch(specs, "f32", steps=24, chunk=12, autotune=False, keep_results=True, steps_per_pass=2)
    for i, s in enumerate(specs):
        _, _, u = serving.run_plain(s, "f32", run.steps[i])
        np.testing.assert_array_equal(run.results[i][1], u, err_msg=s.name)


def _deltas(spec, storage, chunk, chunks, steps_per_pass, policy=None, shape=None):
    b = lbm.lbm_batch_create(1 << 30, chunk, 4)
    out = []
    try:
        lbm.lbm_batch_set_steps_per_pass(b, steps_per_pass, 0)
        if shape is not None:
            lbm.lbm_batch_set_shape(b, *shape)
        if policy is not None:
            lbm.lbm_batch_set_policy(b, policy, 1)
        jid = lbm.lbm_batch_submit(b, serving.job_for(spec, storage, 0.0, chunk * chunks))
        for _ in range(chunks):
            lbm.lbm_batch_run_chunk(b)
            st = lbm.lbm_batch_poll(b, jid)
            out.append((st.steps, st.delta))
    finally:
        lbm.lbm_batch_destroy(b)
    return out


@pytest.mark.parametrize("storage", ["f32", "f16sr", "f64"])
def test_convergence_measure_same_bits_in_every_path(storage):
    """The chunk's last batch sweep (lockstep, one step per launch), the last
    single-lattice sweep of a chunk of one job, and the measure kernel (after
    a chunk that ends with a pass, or with persistent workgroups) all take
    the same measure of the same state."""
    spec = workloads.duct(20, 10, 10, (0.04, 0.01, 0.01), 0.8)
    fused_batch = _deltas(spec, storage, 20, 4, 1)
    persistent = _deltas(spec, storage, 20, 4, 1, shape=(256, 1024, 64))
    fused_solo = _deltas(spec, storage, 20, 4, 1, lbm.LBM_BATCH_LARGE_IN_ORDER)
    kernel = _deltas(spec, storage, 20, 4, 2)
    say(f"{storage}: {fused_batch}")
    assert fused_batch == fused_solo == kernel == persistent
    assert all(d > 0 for _, d in fused_batch)


def test_convergence_measure_of_a_mix_same_bits_fused_and_from_the_state():
    """Eleven lattices of all storage forms in one lockstep chunk: the
    measure combined from the last batch sweep's per-wave maxima (tiles of
    many small lattices, lattice ends inside the combining kernel's rounds)
    equals the measure kernel's, taken from the state (persistent grid)."""
    def run(shape):
        b = lbm.lbm_batch_create(4 << 30, 10, 16)
        try:
            lbm.lbm_batch_set_shape(b, *shape)
            ids = _submit_all(b, MIX, 30)
            out = []
            for _ in range(2):
                lbm.lbm_batch_run_chunk(b)
                out.append([lbm.lbm_batch_poll(b, j).delta for j in ids])
            return out
        finally:
            lbm.lbm_batch_destroy(b)
    fused = run((256, 256, 0))
    fused128 = run((128, 256, 0))
    state = run((256, 1024, 64))
    say(f"fused {fused}")
    assert fused == state == fused128
    assert all(d > 0 for row in fused for d in row)
