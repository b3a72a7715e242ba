"""GPU tests of the batch runtime (multi-lattice sweep, admission by HBM
budget, graph-captured chunks, convergence stop, autotuner) and of the FP16
storage form.

Bar: a lattice advanced in a batch is bit-identical to the same lattice
advanced alone with lbm_step (same per-node update), whatever else is in the
batch; the FP16 and batched forms stay within 1e-3 relative L2 of the FP64
velocity field.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_0811_4593_amd import lbm, serving, workloads  # noqa: E402


def say(msg):
    print(msg, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


MIX = [
    (workloads.duct(37, 12, 9, (0.04, 0.01, 0.01), 0.8), "f32"),
    (workloads.duct(16, 16, 16, (0.03, -0.02, 0.01), 1.3), "f16dev"),
    (workloads.couette(8, 4, 20, 0.05, 1.0), "f32"),
    (workloads.duct(70, 9, 5, (0.02, 0.01, -0.015), 0.65), "f16dev"),
    (workloads.all_classes_lattices()[2], "f32"),
    (workloads.duct(21, 11, 13, (0.01, 0.0, 0.02), 1.0), "f64"),
    (workloads.duct(25, 14, 10, (0.035, 0.01, -0.01), 0.9), "f16sr"),
    # rows of whole 128-byte lines: these jobs are stored row-major
    (workloads.duct(32, 10, 7, (0.03, 0.01, 0.005), 0.85), "f32"),
    (workloads.duct(64, 6, 5, (0.02, -0.01, 0.01), 0.75), "f16dev"),
    (workloads.duct(16, 9, 8, (0.04, 0.0, -0.01), 1.1), "f64"),
    (workloads.duct(64, 7, 6, (0.025, 0.01, 0.01), 0.95), "f16sr"),
]


def _submit_all(b, items, steps):
    return [lbm.lbm_batch_submit(b, serving.job_for(s, st, 0.0, steps)) for s, st in items]


def test_batch_equals_alone_bitwise():
    steps = 40
    b = lbm.lbm_batch_create(4 << 30, 10, 16)
    try:
        ids = _submit_all(b, MIX, steps)
        rounds = 0
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            rounds += 1
            if active == 0 and queued == 0:
                break
        assert rounds == steps // 10
        for jid, (spec, st) in zip(ids, MIX):
            s = lbm.lbm_batch_poll(b, jid)
            assert s.state == lbm.LBM_JOB_DONE and s.steps == steps
            rho_b, u_b = lbm.lbm_batch_result(b, jid, spec.nodes)
            _, rho_p, u_p = serving.run_plain(spec, st, steps)
            say(f"{spec.name} {st}: max |du| {np.abs(u_b - u_p).max():.1e}")
            np.testing.assert_array_equal(rho_b, rho_p)
            np.testing.assert_array_equal(u_b, u_p)
    finally:
        lbm.lbm_batch_destroy(b)


@pytest.mark.parametrize("shape", [(256, 256, 0), (128, 256, 0), (256, 1024, 0), (256, 1024, 64), (128, 4096, 3)],
                         ids=lambda s: "x".join(map(str, s)))
def test_every_launch_shape_gives_the_same_bits(shape):
    """One workgroup per tile (tiles dealt to the XCDs in groups) or a
    persistent grid walking the tile list: every job of the mix ends bitwise
    equal to lbm_step alone."""
    steps = 20
    b = lbm.lbm_batch_create(4 << 30, 10, 16)
    try:
        lbm.lbm_batch_set_steps_per_pass(b, 1, 0)  # every step a launch of this shape
        lbm.lbm_batch_set_shape(b, *shape)
        assert lbm.lbm_batch_get_shape(b) == shape
        ids = _submit_all(b, MIX, steps)
        while lbm.lbm_batch_run_chunk(b) != (0, 0):
            pass
        for jid, (spec, st) in zip(ids, MIX):
            _, u_b = lbm.lbm_batch_result(b, jid, spec.nodes)
            _, _, u_p = serving.run_plain(spec, st, steps)
            np.testing.assert_array_equal(u_b, u_p, err_msg=f"{spec.name} {st} shape {shape}")
    finally:
        lbm.lbm_batch_destroy(b)


def test_batch_fp64_job_matches_oracle():
    spec = workloads.duct(14, 9, 7, (0.04, 0.01, 0.01), 0.8)
    steps = 30
    b = lbm.lbm_batch_create(1 << 30, 6, 4)
    try:
        jid = lbm.lbm_batch_submit(b, serving.job_for(spec, "f64", 0.0, steps))
        while lbm.lbm_batch_run_chunk(b) != (0, 0):
            pass
        rho, u = lbm.lbm_batch_result(b, jid, spec.nodes)
    finally:
        lbm.lbm_batch_destroy(b)
    L = oracle.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, bc=spec.bc)
    r_ref, u_ref = L.moments(L.run(L.init(), steps))
    np.testing.assert_allclose(rho, r_ref.ravel(), rtol=1e-12)
    np.testing.assert_allclose(u, u_ref.ravel(), rtol=0, atol=1e-13)


def test_admission_respects_budget_and_results_unchanged():
    # rows of whole 128-byte lines and a node count that is a multiple of 64:
    # both layouts take the same bytes, so lbm_job_bytes is the job's size
    items = [(workloads.duct(64, 20, 20, (0.03, 0.01, 0.0), 0.9), "f32") for _ in range(5)]
    job_bytes = lbm.lbm_job_bytes(serving.job_for(items[0][0], "f32", 0.0, 20))
    budget = 2 * job_bytes + job_bytes // 2  # room for two jobs at a time
    b = lbm.lbm_batch_create(budget, 10, 8)
    try:
        ids = _submit_all(b, items, 20)
        peak = 0
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            used, cap = lbm.lbm_batch_memory(b)
            assert used <= cap
            peak = max(peak, active)
            if active == 0 and queued == 0:
                break
        assert peak <= 2
        _, _, u_p = serving.run_plain(items[0][0], "f32", 20)
        for jid in ids:
            _, u = lbm.lbm_batch_result(b, jid, items[0][0].nodes)
            np.testing.assert_array_equal(u, u_p)
    finally:
        lbm.lbm_batch_destroy(b)


def test_job_too_large_and_invalid_jobs_rejected():
    b = lbm.lbm_batch_create(8 << 20, 10, 4)
    try:
        big = serving.job_for(workloads.duct(128, 64, 64), "f32", 0.0, 10)
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_batch_submit(b, big)
        assert e.value.status == lbm.LBM_ERR_OOM
        bad = serving.job_for(workloads.duct(10, 8, 8), "f32", 0.0, 10)
        bad.tau = 0.5
        with pytest.raises(lbm.LBMError):
            lbm.lbm_batch_submit(b, bad)
        one_face = lbm.make_job(10, 8, 8, 0.8, {4: (0, 0, 0)})
        with pytest.raises(lbm.LBMError):
            lbm.lbm_batch_submit(b, one_face)
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_batch_result(b, 12345, 10)
        assert e.value.status == lbm.LBM_ERR_ARG
    finally:
        lbm.lbm_batch_destroy(b)


def test_convergence_stop_is_deterministic_and_matches_alone():
    spec = workloads.duct(20, 10, 10, (0.04, 0.01, 0.01), 0.8)
    out = []
    for companions in (0, 3):
        b = lbm.lbm_batch_create(2 << 30, 50, 8)
        try:
            jid = lbm.lbm_batch_submit(b, serving.job_for(spec, "f32", 1e-6, 20000))
            for i in range(companions):
                lbm.lbm_batch_submit(b, serving.job_for(workloads.duct(30 + i, 12, 10), "f16dev", 0.0, 400))
            while lbm.lbm_batch_run_chunk(b)[0] > 0:
                pass
            st = lbm.lbm_batch_poll(b, jid)
            rho, u = lbm.lbm_batch_result(b, jid, spec.nodes)
            out.append((st.steps, st.converged, st.delta, u))
        finally:
            lbm.lbm_batch_destroy(b)
    (s0, c0, d0, u0), (s1, c1, d1, u1) = out
    say(f"stopped at step {s0} (delta {d0:.2e}) alone, {s1} in the mix")
    assert c0 == 1 and c1 == 1 and s0 == s1 and s0 < 20000 and d0 < 1e-6
    np.testing.assert_array_equal(u0, u1)
    # and it is the FP32 steady state: compare with the FP64 oracle
    L = oracle.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, bc=spec.bc)
    _, u_ref = L.moments(L.run(L.init(), s0))
    assert rel_l2(u0, u_ref.ravel()) < 1e-5


def test_convergence_measure_against_host_computation():
    """The delta reported after each chunk is max over nodes and components
    of |u(t) - u(t - chunk)| / u_ref (the snapshot starts at zero), here
    recomputed in double on the host from the same lattice run alone."""
    spec = workloads.duct(20, 10, 10, (0.04, 0.01, 0.01), 0.8)
    chunk, chunks = 20, 5
    u_ref = float(np.linalg.norm(spec.bc[0]))
    b = lbm.lbm_batch_create(1 << 30, chunk, 4)
    got = []
    try:
        jid = lbm.lbm_batch_submit(b, serving.job_for(spec, "f32", 0.0, chunk * chunks))
        for _ in range(chunks):
            lbm.lbm_batch_run_chunk(b)
            st = lbm.lbm_batch_poll(b, jid)
            got.append((st.steps, st.delta))
    finally:
        lbm.lbm_batch_destroy(b)
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, 1.0, None, lbm.LBM_STORE_F32, torch.cuda.current_stream())
    try:
        serving.apply_bc(h, spec)
        u_prev = np.zeros(3 * spec.nodes)
        for k, (steps, delta) in enumerate(got):
            lbm.lbm_step(h, chunk)
            u = np.empty(3 * spec.nodes)
            lbm.lbm_moments(h, None, u)
            expect = float(np.abs(u - u_prev).max()) / u_ref
            say(f"chunk {k + 1}: step {steps}, delta {delta:.6e}, host {expect:.6e}")
            assert steps == chunk * (k + 1)
            # the snapshot u(t - chunk) is kept in float: half an ulp of
            # |u| ~ 0.04 over u_ref is 3e-8 in delta
            assert delta == pytest.approx(expect, rel=1e-3, abs=1e-7)
            u_prev = u
    finally:
        lbm.lbm_destroy(h)


def test_autotune_picks_a_shape_and_results_do_not_change():
    items = MIX[:4]
    b = lbm.lbm_batch_create(4 << 30, 10, 8)
    try:
        ids = _submit_all(b, items, 60)
        shape = lbm.lbm_batch_autotune(b, 2)
        say(f"autotuned shape {shape}")
        assert shape[0] in (128, 256) and shape[1] in (256, 512, 1024)
        assert shape[2] == 0 or shape[1] == 1024  # one workgroup per tile, or a persistent grid
        while lbm.lbm_batch_run_chunk(b) != (0, 0):
            pass
        for jid, (spec, st) in zip(ids, items):
            s = lbm.lbm_batch_poll(b, jid)
            _, u_b = lbm.lbm_batch_result(b, jid, spec.nodes)
            _, _, u_p = serving.run_plain(spec, st, s.steps)
            np.testing.assert_array_equal(u_b, u_p)
    finally:
        lbm.lbm_batch_destroy(b)


def test_fp16_and_fp32_forms_against_fp64_velocity():
    # FP16 scaled-deviation storage with FP32 arithmetic, and FP32 storage,
    # against the FP64 form (parity-pinned to the oracle) on a duct run until
    # the velocity is steady: relative L2 <= 1e-3 (FP16), <= 1e-5 (FP32).
    spec = workloads.duct(48, 24, 24, (0.04, 0.01, 0.01), 0.8)
    steps = 4000
    _, _, u64 = serving.run_plain(spec, "f64", steps)
    _, _, u32 = serving.run_plain(spec, "f32", steps)
    _, _, u16 = serving.run_plain(spec, "f16dev", steps)
    _, _, u16sr = serving.run_plain(spec, "f16sr", steps)
    e32, e16, e16sr = rel_l2(u32, u64), rel_l2(u16, u64), rel_l2(u16sr, u64)
    say(f"rel L2 vs f64: f32 {e32:.2e}, f16dev {e16:.2e}, f16sr {e16sr:.2e}")
    assert e32 <= 1e-5
    assert e16 <= 1e-3
    assert e16sr <= 1e-3


SF, LIO = lbm.LBM_BATCH_SHORTEST_FIRST, lbm.LBM_BATCH_LARGE_IN_ORDER


@pytest.mark.parametrize("policy,lanes,fill", [(SF, 1, 0), (SF, 4, 0), (SF, 4, 6000), (LIO, 4, 6000)],
                         ids=["shortest-1-lane", "shortest-4-lanes", "shortest-shared-launches", "large-in-order"])
def test_serving_loop_small_trace_same_alone_and_in_mix(policy, lanes, fill):
    """The serving loop on a seeded trace of small cubes arriving faster than
    they finish: one lane (one chunk at a time), four lanes with one request
    per lane, four lanes where requests below 6000 nodes share their lane's
    launches, and the serving default (large requests one at a time in
    arrival order, small ones beside them).  Every result equals the request
    run alone, bit for bit; with four lanes chunks run beside each other on
    the device, and with shared launches single launches step several
    requests."""
    trace = workloads.serving_trace(count=12, rate=400.0, seed=3, n_min=12, n_max=28)
    rep = serving.serve_trace(trace, budget_bytes=64 << 20, chunk=50, tol=1e-6, max_steps=1500,
                              max_jobs=4, keep_results=set(range(12)), lanes=lanes, fill_nodes=fill,
                              policy=policy)
    say(f"serve summary lanes={lanes} fill={fill}: {rep.summary()}")
    st = rep.stats
    assert st["lanes"] == lanes
    assert all(x >= 0 for x in rep.latencies)
    assert rep.peak_resident <= 4 and rep.peak_bytes <= 64 << 20
    if lanes > 1:
        assert st["overlapped_chunks"] >= 1 and st["max_lanes_running"] >= 2
    if fill and policy == SF:
        assert st["multi_job_chunks"] >= 1 and st["max_jobs_in_chunk"] >= 2
    for i, r in enumerate(trace):
        _, _, u_alone = serving.run_plain(r.spec, r.storage, rep.steps[i])
        np.testing.assert_array_equal(rep.results[i][1], u_alone)


def test_lanes_lockstep_mix_equals_alone_bitwise():
    """Lockstep with three lanes: the eleven lattices of four storage forms
    are spread over the lanes (several per launch), each lane's chunks run
    beside the others', and every lattice still equals itself run alone."""
    steps = 40
    b = lbm.lbm_batch_create(4 << 30, 10, 16)
    try:
        lbm.lbm_batch_set_lanes(b, 3)
        ids = _submit_all(b, MIX, steps)
        while lbm.lbm_batch_run_chunk(b) != (0, 0):
            pass
        st = lbm.lbm_batch_get_stats(b)
        say(f"lockstep lanes stats {st}")
        assert st["lanes"] == 3 and st["multi_job_chunks"] >= 1
        for jid, (spec, storage) in zip(ids, MIX):
            assert lbm.lbm_batch_poll(b, jid).steps == steps
            rho_b, u_b = lbm.lbm_batch_result(b, jid, spec.nodes)
            _, rho_p, u_p = serving.run_plain(spec, storage, steps)
            np.testing.assert_array_equal(rho_b, rho_p)
            np.testing.assert_array_equal(u_b, u_p)
    finally:
        lbm.lbm_batch_destroy(b)


def test_small_requests_run_beside_a_large_one():
    """Three lanes, shortest remaining work first, one request per lane: two
    small requests that arrive while a large one is running take the idle
    lanes and finish while the large one keeps stepping (with one lane it
    would wait for them); all three equal their runs alone."""
    big = workloads.duct(128, 64, 64, (0.03, 0.01, 0.0), 0.8)
    small = [workloads.duct(16, 16, 16, (0.02, 0.0, 0.01), 0.9), workloads.duct(20, 12, 14, (0.01, 0.01, 0.0), 1.1)]
    b = lbm.lbm_batch_create(1 << 30, 100, 8)
    try:
        lbm.lbm_batch_set_policy(b, lbm.LBM_BATCH_SHORTEST_FIRST, 0)
        lbm.lbm_batch_set_lanes(b, 3)
        jb = lbm.lbm_batch_submit(b, serving.job_for(big, "f32", 0.0, 3000))
        lbm.lbm_batch_run_chunk(b)
        assert lbm.lbm_batch_poll(b, jb).steps == 100
        js = [lbm.lbm_batch_submit(b, serving.job_for(s, "f16sr", 0.0, 800)) for s in small]
        big_steps_when_small_done = None
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            if big_steps_when_small_done is None and \
                    all(lbm.lbm_batch_poll(b, j).state == lbm.LBM_JOB_DONE for j in js):
                big_steps_when_small_done = lbm.lbm_batch_poll(b, jb).steps
            if active == 0 and queued == 0:
                break
        st = lbm.lbm_batch_get_stats(b)
        say(f"large job at {big_steps_when_small_done} steps when the small ones were done; stats {st}")
        assert 200 <= big_steps_when_small_done < 3000
        assert st["overlapped_chunks"] >= 1 and st["max_lanes_running"] >= 2
        for jid, spec, storage, steps in [(jb, big, "f32", 3000)] + [(j, s, "f16sr", 800) for j, s in zip(js, small)]:
            assert lbm.lbm_batch_poll(b, jid).steps == steps
            rho_b, u_b = lbm.lbm_batch_result(b, jid, spec.nodes)
            _, rho_p, u_p = serving.run_plain(spec, storage, steps)
            np.testing.assert_array_equal(rho_b, rho_p)
            np.testing.assert_array_equal(u_b, u_p)
    finally:
        lbm.lbm_batch_destroy(b)


def test_lanes_argument_checks():
    b = lbm.lbm_batch_create(16 << 20, 10, 2)
    try:
        for bad in (0, 9):
            with pytest.raises(lbm.LBMError) as e:
                lbm.lbm_batch_set_lanes(b, bad)
            assert e.value.status == lbm.LBM_ERR_ARG
        lbm.lbm_batch_set_lanes(b, 8)
        lbm.lbm_batch_set_lanes(b, 2)
        assert lbm.lbm_batch_get_stats(b)["lanes"] == 2
        jid = lbm.lbm_batch_submit(b, serving.job_for(workloads.duct(12, 8, 8), "f32", 0.0, 20))
        while lbm.lbm_batch_run_chunk(b) != (0, 0):
            pass
        with pytest.raises(ValueError):
            lbm.lbm_batch_result(b, jid, 12 * 8 * 8 - 1)  # wrong node count: refused before the copy
        rho, u = lbm.lbm_batch_result(b, jid, 12 * 8 * 8)
        assert rho.shape == (768,) and u.shape == (3 * 768,)
    finally:
        lbm.lbm_batch_destroy(b)


def test_large_job_is_not_starved_by_small_ones():
    # Budget: a large job fits only when no small job is resident; three
    # small jobs fit together.  Small jobs may pass the waiting large job
    # during its first four chunks at the head of the queue, then queue
    # behind it.
    # rows of whole lines and node counts that are multiples of 64: both
    # layouts take the same bytes, so lbm_job_bytes is each job's size
    small = workloads.duct(32, 12, 12)
    large = workloads.duct(64, 24, 18)
    sb = lbm.lbm_job_bytes(serving.job_for(small, "f32", 0.0, 10))
    lb = lbm.lbm_job_bytes(serving.job_for(large, "f32", 0.0, 10))
    assert lb > 3 * sb
    b = lbm.lbm_batch_create(lb + sb // 2, 10, 16)
    try:
        first = lbm.lbm_batch_submit(b, serving.job_for(small, "f32", 0.0, 30))
        big = lbm.lbm_batch_submit(b, serving.job_for(large, "f32", 0.0, 20))
        later = [lbm.lbm_batch_submit(b, serving.job_for(small, "f32", 0.0, 20)) for _ in range(12)]
        admitted = {}
        chunk = 0
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            chunk += 1
            for jid in [first, big] + later:
                if jid not in admitted and lbm.lbm_batch_poll(b, jid).state != lbm.LBM_JOB_QUEUED:
                    admitted[jid] = chunk
            if active == 0 and queued == 0:
                break
            assert chunk < 200
        say(f"large job admitted at chunk {admitted[big]}; small ones at {[admitted[j] for j in later]}")
        assert lbm.lbm_batch_poll(b, big).state == lbm.LBM_JOB_DONE
        passed = [j for j in later if admitted[j] < admitted[big]]
        behind = [j for j in later if admitted[j] > admitted[big]]
        assert passed and behind                      # some passed it, the rest waited
        assert max(admitted[j] for j in passed) <= 4  # only during its first four chunks
        rho_l, u_l = lbm.lbm_batch_result(b, big, large.nodes)
        with pytest.raises(lbm.LBMError) as e:        # a result can be taken once
            lbm.lbm_batch_result(b, big, large.nodes)
        assert e.value.status == lbm.LBM_ERR_ARG
    finally:
        lbm.lbm_batch_destroy(b)
    _, _, u_alone = serving.run_plain(large, "f32", 20)
    np.testing.assert_array_equal(u_l, u_alone)


def test_result_of_an_unfinished_job_is_refused():
    b = lbm.lbm_batch_create(256 << 20, 10, 4)
    try:
        jid = lbm.lbm_batch_submit(b, serving.job_for(workloads.duct(20, 10, 10), "f32", 0.0, 40))
        lbm.lbm_batch_run_chunk(b)
        assert lbm.lbm_batch_poll(b, jid).state == lbm.LBM_JOB_RUNNING
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_batch_result(b, jid, 2000)
        assert e.value.status == lbm.LBM_ERR_STATE
    finally:
        lbm.lbm_batch_destroy(b)  # destroying a batch with a resident job is fine


def test_shortest_first_policy_order_and_results():
    """LBM_BATCH_SHORTEST_FIRST with fill_nodes 0 steps one job per chunk, the
    one with the least remaining work: the two small jobs finish before the
    large one takes a step; every result equals the lattice run alone."""
    big = workloads.duct(48, 24, 20, (0.03, 0.01, 0.0), 0.8)
    small = [workloads.duct(10, 8, 6, (0.02, 0.0, 0.01), 0.9), workloads.duct(12, 6, 7, (0.01, 0.01, 0.0), 1.1)]
    b = lbm.lbm_batch_create(256 << 20, 10, 8)
    try:
        lbm.lbm_batch_set_policy(b, lbm.LBM_BATCH_SHORTEST_FIRST, 0)
        jb = lbm.lbm_batch_submit(b, serving.job_for(big, "f32", 0.0, 60))
        js = [lbm.lbm_batch_submit(b, serving.job_for(s, "f16sr", 0.0, 40)) for s in small]
        small_done_first = None
        total_before = 0
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            big_steps = lbm.lbm_batch_poll(b, jb).steps
            ss = [lbm.lbm_batch_poll(b, j) for j in js]
            total = big_steps + sum(st.steps for st in ss)
            assert total - total_before == 10  # one job per chunk, one chunk of steps
            total_before = total
            if small_done_first is None and all(st.state == lbm.LBM_JOB_DONE for st in ss):
                small_done_first = big_steps == 0
            if active == 0 and queued == 0:
                break
        assert small_done_first, "the large job stepped before the small ones were done"
        for jid, spec, st, steps in [(jb, big, "f32", 60)] + [(j, s, "f16sr", 40) for j, s in zip(js, small)]:
            assert lbm.lbm_batch_poll(b, jid).steps == steps
            rho_b, u_b = lbm.lbm_batch_result(b, jid, spec.nodes)
            _, rho_p, u_p = serving.run_plain(spec, st, steps)
            np.testing.assert_array_equal(rho_b, rho_p)
            np.testing.assert_array_equal(u_b, u_p)
    finally:
        lbm.lbm_batch_destroy(b)


def test_shortest_first_does_not_starve_a_large_job():
    """A large job left out for 50 chunks in a row is stepped anyway."""
    big = workloads.duct(40, 20, 16)
    small = workloads.duct(8, 8, 8)
    b = lbm.lbm_batch_create(256 << 20, 10, 4)
    try:
        lbm.lbm_batch_set_policy(b, lbm.LBM_BATCH_SHORTEST_FIRST, 0)
        jb = lbm.lbm_batch_submit(b, serving.job_for(big, "f32", 0.0, 20))
        js = lbm.lbm_batch_submit(b, serving.job_for(small, "f32", 0.0, 2000))
        for chunk in range(52):
            lbm.lbm_batch_run_chunk(b)
        assert lbm.lbm_batch_poll(b, jb).steps >= 10  # stepped after 50 skipped chunks
        assert lbm.lbm_batch_poll(b, js).steps >= 500
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            if active == 0 and queued == 0:
                break
        assert lbm.lbm_batch_poll(b, jb).steps == 20 and lbm.lbm_batch_poll(b, js).steps == 2000
    finally:
        lbm.lbm_batch_destroy(b)


def test_batch_policy_rejects_unknown_values():
    b = lbm.lbm_batch_create(16 << 20, 10, 2)
    try:
        with pytest.raises(lbm.LBMError) as e:
            lbm.lbm_batch_set_policy(b, 7, 0)
        assert e.value.status == lbm.LBM_ERR_ARG
    finally:
        lbm.lbm_batch_destroy(b)


@pytest.mark.parametrize("storage", ["f64", "f16dev", "f32", "f16sr"])
def test_single_sweep_chunks_every_storage_form(storage):
    """Shortest first with one job per chunk stores jobs row-major with padded
    rows (37 wide: 48 FP64, 64 FP32/FP16 elements) and steps each chunk's job
    with the single-lattice sweep; a duct with velocity faces and a forced
    channel still equal the lattices run alone, bit for bit."""
    duct = workloads.duct(37, 9, 8, (0.03, 0.01, -0.01), 0.85)
    chan = workloads.LatticeSpec(21, 10, 9, 1.0, {4: (0.0, 0.0, 0.0), 5: (0.0, 0.0, 0.0)}, name="forced_channel")
    b = lbm.lbm_batch_create(256 << 20, 10, 4)
    try:
        lbm.lbm_batch_set_policy(b, lbm.LBM_BATCH_SHORTEST_FIRST, 0)
        j1 = lbm.lbm_batch_submit(b, serving.job_for(duct, storage, 0.0, 30))
        job = serving.job_for(chan, storage, 0.0, 40)
        job.force[0], job.force[1] = 1e-5, 2e-6
        j2 = lbm.lbm_batch_submit(b, job)
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            if active == 0 and queued == 0:
                break
        rho_b, u_b = lbm.lbm_batch_result(b, j1, duct.nodes)
        _, rho_p, u_p = serving.run_plain(duct, storage, 30)
        np.testing.assert_array_equal(rho_b, rho_p)
        np.testing.assert_array_equal(u_b, u_p)
        rho_c, u_c = lbm.lbm_batch_result(b, j2, chan.nodes)
        h = lbm.lbm_create(chan.nx, chan.ny, chan.nz, chan.tau, 1.0, None, serving.STORAGE[storage],
                           torch.cuda.current_stream())
        try:
            serving.apply_bc(h, chan)
            lbm.lbm_set_body_force(h, (1e-5, 2e-6, 0.0))
            lbm.lbm_step(h, 40)
            rho, u = np.empty(chan.nodes), np.empty(3 * chan.nodes)
            lbm.lbm_moments(h, rho, u)
        finally:
            lbm.lbm_destroy(h)
        np.testing.assert_array_equal(rho_c, rho)
        np.testing.assert_array_equal(u_c, u)
    finally:
        lbm.lbm_batch_destroy(b)


def test_large_in_order_policy():
    """LBM_BATCH_LARGE_IN_ORDER with three lanes: the two large jobs (at least
    4000 nodes) run one after the other in submission order, the small ones
    beside the first; every result equals the lattice run alone."""
    large = [workloads.duct(24, 16, 14, (0.03, 0.01, 0.0), 0.8), workloads.duct(20, 18, 15, (0.02, 0.0, 0.01), 0.9)]
    small = [workloads.duct(10, 8, 6, (0.02, 0.0, 0.01), 0.9), workloads.duct(12, 6, 7, (0.01, 0.01, 0.0), 1.1)]
    b = lbm.lbm_batch_create(256 << 20, 10, 8)
    try:
        lbm.lbm_batch_set_policy(b, lbm.LBM_BATCH_LARGE_IN_ORDER, 4000)
        lbm.lbm_batch_set_lanes(b, 3)
        jl = [lbm.lbm_batch_submit(b, serving.job_for(s, "f32", 0.0, 200)) for s in large]
        js = [lbm.lbm_batch_submit(b, serving.job_for(s, "f16sr", 0.0, 60)) for s in small]
        small_done_at = None
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            s0, s1 = (lbm.lbm_batch_poll(b, j) for j in jl)
            if s1.steps > 0:  # the second large job starts only after the first is done
                assert s0.state == lbm.LBM_JOB_DONE
            if small_done_at is None and all(lbm.lbm_batch_poll(b, j).state == lbm.LBM_JOB_DONE for j in js):
                small_done_at = s0.steps
            if active == 0 and queued == 0:
                break
        st = lbm.lbm_batch_get_stats(b)
        say(f"first large job at {small_done_at} steps when the small ones were done; stats {st}")
        assert small_done_at < 200 and st["overlapped_chunks"] >= 1
        for jid, spec, storage, steps in [(j, s, "f32", 200) for j, s in zip(jl, large)] + \
                [(j, s, "f16sr", 60) for j, s in zip(js, small)]:
            assert lbm.lbm_batch_poll(b, jid).steps == steps
            rho_b, u_b = lbm.lbm_batch_result(b, jid, spec.nodes)
            _, rho_p, u_p = serving.run_plain(spec, storage, steps)
            np.testing.assert_array_equal(rho_b, rho_p)
            np.testing.assert_array_equal(u_b, u_p)
    finally:
        lbm.lbm_batch_destroy(b)
