"""Batch and serving drivers on top of the batch runtime of liblbm.so.

The runtime (admission by HBM budget, device memory pool, multi-lattice
sweep, graph-captured chunks, convergence measure, autotuner) is native; this
module only turns workload descriptions into jobs, replays arrival traces in
real time and collects latencies.  No arithmetic of the method happens here.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm

STORAGE = {"f64": lbm.LBM_STORE_F64, "f32": lbm.LBM_STORE_F32, "f16dev": lbm.LBM_STORE_F16_DEV,
           "f16sr": lbm.LBM_STORE_F16_DEV_SR}


def job_for(spec, storage: str, tol: float = 0.0, max_steps: int = 0):
    return lbm.make_job(spec.nx, spec.ny, spec.nz, spec.tau, spec.bc, STORAGE[storage], spec.rho0,
                        tol=tol, max_steps=max_steps, pressure=getattr(spec, "pressure", None))


def percentile(values, q):
    return float(np.percentile(np.asarray(values, dtype=float), q)) if len(values) else float("nan")


@dataclass
class BatchRun:
    seconds: float
    steps: dict                # job index -> steps taken
    results: dict              # job index -> (rho, u)
    shape: tuple
    node_updates: float = 0.0


def run_batch(specs, storage="f32", steps=2000, chunk=100, budget_bytes=None, autotune=True, trial_steps=4,
              stream=None, keep_results=True, steps_per_pass=None):
    """Run every spec as one job of a batch for `steps` steps (no early stop).
    Returns the wall time from the first chunk to the last retirement."""
    jobs = [job_for(s, storage, 0.0, steps) for s in specs]
    need = sum(lbm.lbm_job_bytes(j) for j in jobs)
    budget = budget_bytes or int(need * 1.05) + (64 << 20)
    b = lbm.lbm_batch_create(budget, chunk, max(len(jobs), 1), stream)
    try:
        if steps_per_pass is not None:
            lbm.lbm_batch_set_steps_per_pass(b, steps_per_pass, 0)
        ids = [lbm.lbm_batch_submit(b, j) for j in jobs]
        t0 = time.perf_counter()
        shape = lbm.lbm_batch_autotune(b, trial_steps) if autotune else lbm.lbm_batch_get_shape(b)
        while True:
            active, queued = lbm.lbm_batch_run_chunk(b)
            if active == 0 and queued == 0:
                break
        seconds = time.perf_counter() - t0
        out_steps, results = {}, {}
        updates = 0.0
        for i, (jid, s) in enumerate(zip(ids, specs)):
            st = lbm.lbm_batch_poll(b, jid)
            out_steps[i] = st.steps
            updates += float(st.steps) * s.nodes
            rho, u = lbm.lbm_batch_result(b, jid, s.nodes)
            if keep_results:
                results[i] = (rho, u)
        return BatchRun(seconds, out_steps, results, shape, updates)
    finally:
        lbm.lbm_batch_destroy(b)


def apply_bc(h, spec):
    """Set the faces of a workload description on a lattice handle."""
    pressure = getattr(spec, "pressure", {}) or {}
    for face, v in spec.bc.items():
        if face not in pressure:
            lbm.lbm_set_velocity_bc(h, face, v)
    for face, r in pressure.items():
        lbm.lbm_set_pressure_bc(h, face, r, spec.bc.get(face))


def _host_array(n):
    """A float64 host array in page-locked memory when a GPU runtime is there
    (the batch runtime holds its results in page-locked memory too, so both
    sides of a comparison copy at the same speed), else ordinary memory."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.empty(n, dtype=torch.float64, pin_memory=True).numpy()
    except ImportError:
        pass
    return np.empty(n)


def run_plain(spec, storage="f32", steps=2000, stream=None, launch=None):
    """One lattice with plain lbm_step launches in the row-major layout (the
    faster one for a single lattice); returns (seconds, rho, u)."""
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, STORAGE[storage], stream)
    try:
        apply_bc(h, spec)
        lbm.lbm_set_layout(h, lbm.LBM_LAYOUT_ROW_MAJOR)
        if launch:
            lbm.lbm_set_launch(h, *launch)
        rho = _host_array(spec.nodes)
        u = _host_array(3 * spec.nodes)
        t0 = time.perf_counter()
        lbm.lbm_step(h, steps)
        lbm.lbm_moments(h, rho, u)  # synchronizes
        return time.perf_counter() - t0, rho, u
    finally:
        lbm.lbm_destroy(h)


@dataclass
class ServeReport:
    latencies: list = field(default_factory=list)   # seconds, per request in id order
    steps: list = field(default_factory=list)
    converged: list = field(default_factory=list)
    seconds: float = 0.0
    results: dict = field(default_factory=dict)
    peak_resident: int = 0
    peak_bytes: int = 0
    stats: dict = field(default_factory=dict)  # lbm_batch_get_stats at the end (served runs)

    @property
    def solves_per_s(self):
        return len(self.latencies) / self.seconds if self.seconds > 0 else float("nan")

    def summary(self):
        out = {"requests": len(self.latencies), "seconds": round(self.seconds, 3),
               "solves_per_s": round(self.solves_per_s, 3),
               "p50_s": round(percentile(self.latencies, 50), 4), "p99_s": round(percentile(self.latencies, 99), 4),
               "converged": int(sum(self.converged)), "peak_resident": self.peak_resident,
               "peak_bytes": self.peak_bytes}
        if self.stats:
            out["batch_stats"] = dict(self.stats)
        return out


SERVE_LANES = 4  # concurrent lanes of the serving loop (HIP's default of 4 hardware queues per process)
SERVE_LARGE_NODES = 1 << 18  # requests of at least 64^3 nodes run one at a time, in arrival order


def serve_trace(trace, budget_bytes, chunk=100, tol=1e-6, max_steps=20000, max_jobs=256, shape=None,
                keep_results=(), stream=None, progress=None, policy=lbm.LBM_BATCH_LARGE_IN_ORDER,
                fill_nodes=SERVE_LARGE_NODES, lanes=SERVE_LANES):
    """Replay `trace` (workloads.Request list, sorted by arrival) in real time:
    each request is submitted at its arrival time; between submissions the
    batch runs chunks, admitting queued requests as slots and memory free up
    (continuous batching).  With `lanes` > 1 the chunks of up to `lanes`
    groups of requests run on the device at the same time (lbm_batch_set_lanes),
    so a request that arrives while others run starts at once beside them;
    `policy` forms the groups (lbm_batch_set_policy): by default large
    requests (at least fill_nodes nodes) one at a time in arrival order and
    small ones beside them on the other lanes; with shortest remaining work
    first, a request below fill_nodes nodes shares its lane's launches with
    other small ones up to fill_nodes nodes.  Latency = completion time - arrival
    time.  progress(done, total), if given, is called after every
    completion."""
    b = lbm.lbm_batch_create(budget_bytes, chunk, max_jobs, stream)
    rep = ServeReport()
    try:
        lbm.lbm_batch_set_policy(b, policy, fill_nodes)
        lbm.lbm_batch_set_lanes(b, lanes)
        if shape:
            lbm.lbm_batch_set_shape(b, *shape)
        nreq = len(trace)
        job_of = {}
        done_at = [None] * nreq
        steps = [0] * nreq
        conv = [0] * nreq
        nxt = 0
        t0 = time.perf_counter()
        outstanding = 0
        while nxt < nreq or outstanding:
            now = time.perf_counter() - t0
            while nxt < nreq and trace[nxt].arrival <= now:
                r = trace[nxt]
                job_of[lbm.lbm_batch_submit(b, job_for(r.spec, r.storage, tol, max_steps))] = nxt
                nxt += 1
                outstanding += 1
            if outstanding == 0:
                time.sleep(max(0.0, trace[nxt].arrival - (time.perf_counter() - t0)))
                continue
            active, _ = lbm.lbm_batch_run_chunk(b)
            used, _ = lbm.lbm_batch_memory(b)
            rep.peak_resident = max(rep.peak_resident, active)
            rep.peak_bytes = max(rep.peak_bytes, used)
            t_now = time.perf_counter() - t0
            for jid in list(job_of):
                st = lbm.lbm_batch_poll(b, jid)
                if st.state == lbm.LBM_JOB_DONE:
                    i = job_of.pop(jid)
                    done_at[i] = t_now
                    steps[i] = st.steps
                    conv[i] = st.converged
                    # the moments are on the host (page-locked) since the
                    # chunk retired the job; copy out only the kept ones
                    if i in keep_results:
                        rep.results[i] = lbm.lbm_batch_result(b, jid, trace[i].spec.nodes)
                    else:
                        lbm.lbm_batch_result(b, jid, None)
                    outstanding -= 1
                    if progress:
                        progress(sum(d is not None for d in done_at), nreq)
        rep.seconds = time.perf_counter() - t0
        rep.latencies = [done_at[i] - trace[i].arrival for i in range(nreq)]
        rep.steps = steps
        rep.converged = conv
        rep.stats = lbm.lbm_batch_get_stats(b)
        return rep
    finally:
        lbm.lbm_batch_destroy(b)


def replay_one_at_a_time(trace, steps, stream=None, progress=None):
    """Baseline: the same arrival trace served first-come first-served, one
    request at a time with plain lbm_step launches, each for the step count
    the batched run needed for it.  Returns a ServeReport."""
    rep = ServeReport()
    t0 = time.perf_counter()
    free_at = 0.0
    lat = []
    for r, n in zip(trace, steps):
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        run_plain(r.spec, r.storage, n, stream)
        free_at = time.perf_counter() - t0
        lat.append(free_at - r.arrival)
        if progress:
            progress(len(lat), len(trace))
    rep.seconds = time.perf_counter() - t0
    rep.latencies = lat
    rep.steps = list(steps)
    rep.converged = [0] * len(lat)
    return rep
