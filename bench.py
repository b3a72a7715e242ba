#!/usr/bin/env python3
"""Throughput of the fused D3Q19 sweep on one MI355X.

Workload: the 1024 x 512 x 512 duct (no-slip on-site walls on the y and z
faces, on-site velocity inlet and outlet (0.04, 0.01, 0.01) on the x faces,
tau = 0.8, FP32 storage), initial state at rest, synthetic.  A step is one
update of all 2^28 nodes (pull streaming, boundary rules, BGK collision);
by default two steps run per pass over HBM (lbm_set_steps_per_pass: one
launch of the two-step kernel per pair of steps, bitwise the state of two
single sweeps; --steps-per-pass 1: one single sweep per step).  The
populations are stored row-major (the 19 populations of each x-row
together; --layout pop: population-major), and the lattice's two buffers
are chosen by lbm_tune_placement from a pool of 8 allocations (its trial
steps are real, untimed steps; --placement 0 keeps the lattice's own).  Then
W untimed warm-up steps, then exactly K timed steps bracketed by device
synchronisation.

Printed: one JSON line with MLUPS (the value), the roofline object for the
timed kernel (algorithmic bytes per launch / average launch duration
measured with HIP events on the launch stream), the bandwidth probes of the
same buffers, the CPU oracle timed on a bounded sample of the same workload,
and the systems forms (storage precision, batching, serving) at their own
configured sizes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

_ROOT = os.path.dirname(os.path.abspath(__file__))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
METRIC = "D3Q19 MLUPS & % HBM roofline; batched solves/s, p50/p99 at ≤1e-3 L2 err"
COUNTERS_FILE = os.path.join(_ROOT, "profiles", "sweep2_f32_duct_1024x512x512_counters.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("d3q19.hpp", "node_update.hpp", "lbm_kernels.hip", "lbm_sweep2.hip", "sweep2_box.hpp",
                 "lbm_internal.hpp"):
        with open(os.path.join(_ROOT, "paper_0811_4593_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(launch, storage, layout, steps_per_launch=1, pass_args=None):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source, launch shape and pass; else
    None."""
    try:
        with open(COUNTERS_FILE) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_hash") != kernel_source_hash() or c.get("launch") != list(launch) \
            or c.get("storage") != storage or c.get("layout", "pop") != layout \
            or c.get("steps_per_launch", 1) != steps_per_launch \
            or (pass_args is not None and c.get("pass", [1, 0, 0]) != list(pass_args)):
        return None
    return c.get("hbm_bytes_per_launch")


def _counter_means(path, counter):
    import csv
    acc = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def ingest_counters(args):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the sweep kernel, each
    scaled by the ratio of the known byte count of the contiguous-copy probe
    (the 19 P elements of a buffer read and written) to what the same counter
    reads for it."""
    from paper_0811_4593_amd import lbm

    fetch = _counter_means(args.ingest_counters[0], "FETCH_SIZE")
    write = _counter_means(args.ingest_counters[1], "WRITE_SIZE")
    storage = {"f32": lbm.LBM_STORE_F32, "f64": lbm.LBM_STORE_F64, "f16dev": lbm.LBM_STORE_F16_DEV,
               "f16sr": lbm.LBM_STORE_F16_DEV_SR}[args.storage]
    N = args.nx * args.ny * args.nz
    # the probe copies the whole buffer (its size in the layout), in 16-byte units
    layout = {"pop": lbm.LBM_LAYOUT_POPULATION_MAJOR, "rows": lbm.LBM_LAYOUT_ROW_MAJOR}[args.layout]
    buf_elems = lbm.lbm_buffer_elements(args.nx, args.ny, args.nz, storage, layout)
    copy_kib = (buf_elems * lbm.lbm_element_bytes(storage) // 16 * 16) / 1024.0

    def pick(d, frag):
        ks = [k for k in d if frag in k]
        assert len(ks) == 1, (frag, list(d))
        return ks[0], d[ks[0]]

    # the timed kernel: the two-step pass if the run used it, else the full
    # single sweep (COPY = false, EXT = false)
    frag = "sweep2_kernel" if any("sweep2_kernel" in k for k in fetch) else ", false, false>("
    steps_per_launch = 2 if frag == "sweep2_kernel" else 1
    sweep_name, f_sweep = pick(fetch, frag)
    _, w_sweep = pick(write, frag)
    _, f_copy = pick(fetch, "copy_probe_kernel")
    _, w_copy = pick(write, "copy_probe_kernel")
    fs, ws = copy_kib / f_copy, copy_kib / w_copy
    launch = [int(t) for t in args.launch.split(",")] if args.launch else None
    rec = {
        "kernel": sweep_name,
        "kernel_source_hash": kernel_source_hash(),
        "storage": args.storage,
        "layout": args.layout,
        "launch": launch,
        "lattice": [args.nx, args.ny, args.nz],
        "fetch_kib_per_dispatch": f_sweep,
        "write_kib_per_dispatch": w_sweep,
        "copy_probe_fetch_kib": f_copy,
        "copy_probe_write_kib": w_copy,
        "copy_probe_known_kib": copy_kib,
        "fetch_scale": fs,
        "write_scale": ws,
        "steps_per_launch": steps_per_launch,
        "pass": [args.steps_per_pass, args.zplanes, args.tile_rows],  # as given to bench.py
        "hbm_bytes_per_launch": (f_sweep * fs + w_sweep * ws) * 1024.0,
        "algorithmic_bytes_per_launch": 2 * 19 * N * lbm.lbm_element_bytes(storage) * steps_per_launch,
        "command": args.counters_command,
    }
    out = getattr(args, "counters_out", "") or COUNTERS_FILE
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))


def cpu_baseline(spec_full, budget_s: float):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the workload:
    the same duct set-up at 256 x 128 x 128 (1/64 of the nodes), stepped until
    `budget_s` seconds have passed (at least 2 steps)."""
    import oracle
    from paper_0811_4593_amd import workloads

    s = workloads.duct(256, 128, 128, spec_full.bc[0], spec_full.tau)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    L = oracle.Lattice(s.nx, s.ny, s.nz, s.tau, bc=s.bc)
    f = L.init()
    f = L.step(f, nthreads=threads)  # first touch of the buffers, untimed
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = L.step(f, nthreads=threads)
        steps += 1
        el = time.perf_counter() - t0
        if (el >= budget_s and steps >= 2) or steps >= 2000:
            break
    mlups = s.nodes * steps / el / 1e6
    # the same sample on one thread, for a third of the budget
    steps1 = 0
    t0 = time.perf_counter()
    while True:
        f = L.step(f, nthreads=1)
        steps1 += 1
        el1 = time.perf_counter() - t0
        if (el1 >= budget_s / 3 and steps1 >= 1) or steps1 >= 500:
            break
    mlups1 = s.nodes * steps1 / el1 / 1e6
    # the 16 x 16 x 32 Couette flow, 2000 steps in FP64, in full
    c = workloads.couette(16, 16, 32, 0.05, 1.0)
    Lc = oracle.Lattice(c.nx, c.ny, c.nz, c.tau, bc=c.bc)
    fc = Lc.init()
    t0 = time.perf_counter()
    for _ in range(2000):
        fc = Lc.step(fc, nthreads=threads)
    el_c = time.perf_counter() - t0
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": threads, "cpu_model": cpu_model(), "kind": "oracle",
            "single_thread_value": round(mlups1, 3), "couette_16x16x32_2000_steps_s": round(el_c, 3),
            "sample": f"duct {s.nx}x{s.ny}x{s.nz} (same boundary set-up, 1/64 of the nodes), FP64, "
                      f"{steps} steps in {el:.1f} s on {threads} threads; effective {mlups * 304 / 1e3:.2f} GB/s "
                      f"at 304 B/node; on 1 thread {steps1} steps in {el1:.1f} s"}


def _device_rel_l2(u, ref):
    import torch
    return float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(ref))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def form_precision(args, steps=20000):
    """Storage precision on the 512x256x256 duct: FP16 scaled deviations (FP32
    arithmetic) and FP32 storage against the FP64 form (the GPU FP64 path is
    parity-pinned to the CPU oracle at 1e-12 per step) after the same number of
    steps; MLUPS of each form on the same lattice, including the FP64
    mass/momentum reductions taken every 100 steps to monitor the density
    drift (its mass at the first and last reduction is reported)."""
    import torch

    from paper_0811_4593_amd import lbm, workloads

    spec = workloads.precision_duct()
    N = spec.nodes
    res, fields = {}, {}
    for name, st in (("f64", lbm.LBM_STORE_F64), ("f32", lbm.LBM_STORE_F32), ("f16dev", lbm.LBM_STORE_F16_DEV),
                     ("f16sr", lbm.LBM_STORE_F16_DEV_SR)):
        stream = torch.cuda.current_stream()
        h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, st, stream)
        try:
            for face, v in spec.bc.items():
                lbm.lbm_set_velocity_bc(h, face, v)
            lbm.lbm_set_layout(h, lbm.LBM_LAYOUT_ROW_MAJOR)
            # launch shape and buffer placement picked on real steps; they count towards the run
            shape = lbm.lbm_autotune(h, 4)
            tried, ms0, ms1 = lbm.lbm_tune_placement(h, 6, 1)
            done = lbm.lbm_get_step(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            masses = []
            left = steps - done
            while left > 0:
                n = min(100, left)
                lbm.lbm_step(h, n)
                left -= n
                mass, mom = lbm.lbm_totals(h)  # FP64 reduction (synchronizes)
                masses.append(mass)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            u = torch.empty(3 * N, dtype=torch.float64, device="cuda")
            lbm.lbm_moments(h, None, u, dst_on_device=True)
        finally:
            lbm.lbm_destroy(h)
        fields[name] = u
        res[name] = {"MLUPS": round(N * (steps - done) / sec / 1e6, 1),
                     "GBs": round(N * (steps - done) / sec * 2 * 19 * lbm.lbm_element_bytes(st) / 1e9, 1),
                     "launch": list(shape), "layout": "row-major",
                     "placement_ms_per_step": [round(ms0, 4), round(ms1, 4)],
                     "mass": mass, "momentum": [float(x) for x in mom],
                     "reductions": len(masses), "mass_first_last": [masses[0], masses[-1]]}
        print(f"precision form: {name} done in {sec:.1f} s", file=sys.stderr, flush=True)
    for name in ("f32", "f16dev", "f16sr"):
        res[name]["rel_L2_u_vs_f64"] = _device_rel_l2(fields[name], fields["f64"])
    return {"form": "precision", "workload": f"duct {spec.nx}x{spec.ny}x{spec.nz}, inlet/outlet (0.04,0.01,0.01), "
            f"no-slip y/z walls, tau {spec.tau}", "steps": steps, "results": res,
            "f16_over_f32_MLUPS": round(res["f16dev"]["MLUPS"] / res["f32"]["MLUPS"], 3),
            "f16sr_over_f32_MLUPS": round(res["f16sr"]["MLUPS"] / res["f32"]["MLUPS"], 3)}


def form_batch(args, steps=2000):
    """64 seeded uneven ducts (Nx ~ U{32..256}, Ny, Nz ~ U{16..128}, oblique
    inflow |u| ~ U[0.01, 0.05], tau ~ U[0.6, 1.5], FP32) in one batch:
    autotuned shape, 100-step graph chunks, 2000 steps each; against the same
    64 lattices run one after another with plain launches."""
    from paper_0811_4593_amd import serving, workloads

    specs = workloads.batch_ducts(64, seed=0)
    # 16 real steps per autotuner candidate: 4 left the pick between
    # near-equal shapes to noise
    run = serving.run_batch(specs, "f32", steps=steps, chunk=100, autotune=True, trial_steps=16, keep_results=True)
    print(f"batch form: batched run {run.seconds:.2f} s", file=sys.stderr, flush=True)
    seq_s, worst = 0.0, 0.0
    seq_updates = 0.0
    for i, s in enumerate(specs):
        sec, _, u = serving.run_plain(s, "f32", run.steps[i])
        seq_s += sec
        seq_updates += run.steps[i] * s.nodes
        ub = run.results[i][1]
        worst = max(worst, float(np.linalg.norm(ub - u) / np.linalg.norm(u)))
    nodes = sum(s.nodes for s in specs)
    return {"form": "batch", "lattices": len(specs), "nodes": nodes, "steps_each": sorted(set(run.steps.values())),
            "shape": {"block_x": run.shape[0], "tile_nodes": run.shape[1], "grid": run.shape[2]},
            "batched": {"seconds": round(run.seconds, 3), "MLUPS": round(run.node_updates / run.seconds / 1e6, 1),
                        "solves_per_s": round(len(specs) / run.seconds, 2)},
            "sequential_plain": {"seconds": round(seq_s, 3), "MLUPS": round(seq_updates / seq_s / 1e6, 1),
                                 "solves_per_s": round(len(specs) / seq_s, 2)},
            "speedup": round(seq_s / run.seconds, 2),
            "max_rel_L2_u_batched_vs_plain": worst, "bitwise_equal_to_plain": worst == 0.0}


def form_serve(args, requests=40):
    """Serving: seeded Poisson arrivals of cubic ducts, N log-uniform in
    [16, 256], oblique inflow |u| ~ U[0.01, 0.05], tau ~ U[0.6, 1.5], FP16 or
    FP32 per request, each run until the relative velocity change over 100
    steps is below 1e-6 or 20000 steps.  A calibration pass submits the first
    requests at once to measure saturated solves/s; the timed trace arrives at
    0.7 times that rate.  Baseline: the same trace served one request at a time
    with plain launches."""
    import torch

    from paper_0811_4593_amd import lbm, serving, workloads

    free, total = torch.cuda.mem_get_info()
    budget = int(min(free * 0.8, 200e9))
    calib = workloads.serving_trace(count=12, rate=1e9, seed=1)
    policy = {"shortest": lbm.LBM_BATCH_SHORTEST_FIRST, "large-in-order": lbm.LBM_BATCH_LARGE_IN_ORDER}[
        args.serve_policy]
    rep_c = serving.serve_trace(calib, budget, chunk=100, tol=1e-6, max_steps=20000, max_jobs=512,
                                fill_nodes=args.serve_fill, lanes=args.serve_lanes, policy=policy)
    sat = rep_c.solves_per_s
    print(f"serve form: calibration {rep_c.summary()}", file=sys.stderr, flush=True)
    rate = 0.7 * sat
    trace = workloads.serving_trace(count=requests, rate=rate, seed=1)
    def progress(what):
        def report(done, total):
            if done % 10 == 0 or done == total:
                print(f"serve form: {what} {done}/{total}", file=sys.stderr, flush=True)
        return report

    rep = serving.serve_trace(trace, budget, chunk=100, tol=1e-6, max_steps=20000, max_jobs=512,
                              fill_nodes=args.serve_fill, lanes=args.serve_lanes, policy=policy,
                              progress=progress("served"))
    print(f"serve form: served {rep.summary()}", file=sys.stderr, flush=True)
    base = serving.replay_one_at_a_time(trace, rep.steps, progress=progress("one at a time"))
    print(f"serve form: one-at-a-time {base.summary()}", file=sys.stderr, flush=True)
    nodes = [r.spec.nodes for r in trace]
    sv, oa = rep.summary(), base.summary()
    if args.serve_policy == "shortest":
        pol = (f"{args.serve_lanes} lanes, shortest remaining work first, requests below {args.serve_fill} nodes "
               f"share launches up to {args.serve_fill} nodes")
    else:
        pol = (f"{args.serve_lanes} lanes: requests of at least {args.serve_fill} nodes one at a time in arrival "
               f"order, smaller ones beside them, shortest remaining work first")
    return {"form": "serve", "policy": pol,
            "requests": len(trace), "rate_per_s": round(rate, 4),
            "calibration_solves_per_s": round(sat, 4), "budget_bytes": budget,
            "mean_nodes": float(np.mean(nodes)), "storage_f16_share": float(np.mean([r.storage == "f16sr" for r in trace])),
            "served": sv, "one_at_a_time": oa,
            "p50_served_over_one_at_a_time": round(sv["p50_s"] / oa["p50_s"], 3),
            "p99_served_over_one_at_a_time": round(sv["p99_s"] / oa["p99_s"], 3),
            "steps_mean": float(np.mean(rep.steps)), "converged": int(sum(rep.converged))}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16dev", "f16sr"])
    ap.add_argument("--launch", default=None, help="block_x,nodes_per_thread,xcd_remap (default: library's)")
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--nz", type=int, default=512)
    ap.add_argument("--probe-reps", type=int, default=10)
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shape with lbm_autotune during the warm-up (default: the library's "
                         "default shape, the fastest measured on this workload)")
    ap.add_argument("--placement", type=int, default=8,
                    help="buffers in the pool of lbm_tune_placement before the warm-up (the sweep's speed depends "
                         "on where its two buffers lie; its trial steps are real, untimed steps); < 2: off")
    ap.add_argument("--layout", default="rows", choices=["pop", "rows"],
                    help="population layout of the device buffers: population-major (k*P + n) or row-major "
                         "(the 19 populations of each x-row together)")
    ap.add_argument("--steps-per-pass", type=int, default=2, choices=[1, 2],
                    help="time steps per pass over HBM (lbm_set_steps_per_pass; 2: two steps per read and write "
                         "of the state, the fastest measured on this workload)")
    ap.add_argument("--zplanes", type=int, default=32, help="z-planes per workgroup of the two-step pass (0: 64)")
    ap.add_argument("--tile-rows", type=int, default=0, help="interior rows of the two-step tiles (0: the form's default, 5 or 12)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE) "
                         "into the committed counters file and exit")
    ap.add_argument("--counters-command", default="", help="the rocprofv3 command lines, for the record")
    ap.add_argument("--counters-out", default="",
                    help="file the summary goes to (default: the counters file the bench line reads)")
    ap.add_argument("--form", choices=["precision", "batch", "serve"], default=None,
                    help="measure one of the systems forms instead of the roofline run (see form_* below)")
    ap.add_argument("--requests", type=int, default=40, help="--form serve: requests in the timed trace")
    ap.add_argument("--precision-steps", type=int, default=20000,
                    help="precision leg: steps of the 512x256x256 duct in every storage form (not --steps)")
    ap.add_argument("--batch-steps", type=int, default=2000, help="batch leg: steps of each of the 64 ducts")
    ap.add_argument("--serve-requests", type=int, default=20,
                    help="serving leg of the default run: requests of the seeded trace (bounded so that the "
                         "whole run stays within a few minutes; --form serve --requests N for longer traces)")
    ap.add_argument("--legs", default="precision,batch,serve",
                    help="systems forms measured after the roofline run and reported under 'forms' "
                         "(comma list of precision, batch, serve; empty: none)")
    ap.add_argument("--serve-fill", type=int, default=1 << 18,
                    help="serve form: with large-in-order, the node count from which a request is large; with "
                         "shortest, requests below it share their lane's launches up to it (0: one per lane)")
    ap.add_argument("--serve-policy", default="large-in-order", choices=["shortest", "large-in-order"],
                    help="serve form: how the lanes are filled (lbm_batch_set_policy)")
    ap.add_argument("--serve-lanes", type=int, default=4,
                    help="serve form: lanes (concurrent chunk streams) of the batch runtime")
    args = ap.parse_args()

    if args.ingest_counters:
        ingest_counters(args)
        return
    if args.form:
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        if args.form == "precision":
            out = form_precision(args, args.precision_steps)
        elif args.form == "batch":
            out = form_batch(args, args.batch_steps)
        else:
            out = form_serve(args, args.requests)
        print(json.dumps(out), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the single-lattice path "
              "does not shard across GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_0811_4593_amd import lbm, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    storage = {"f32": lbm.LBM_STORE_F32, "f64": lbm.LBM_STORE_F64, "f16dev": lbm.LBM_STORE_F16_DEV,
               "f16sr": lbm.LBM_STORE_F16_DEV_SR}[args.storage]
    ebytes = lbm.lbm_element_bytes(storage)
    spec = workloads.duct(args.nx, args.ny, args.nz, (0.04, 0.01, 0.01), 0.8)
    N = spec.nodes
    stream = torch.cuda.current_stream()
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, storage, stream)
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        layout = {"pop": lbm.LBM_LAYOUT_POPULATION_MAJOR, "rows": lbm.LBM_LAYOUT_ROW_MAJOR}[args.layout]
        lbm.lbm_set_layout(h, layout)
        tuned = False
        if args.launch:
            lbm.lbm_set_launch(h, *[int(t) for t in args.launch.split(",")])
        elif args.autotune:
            # the autotuner's trial steps are real, untimed steps (part of the warm-up)
            lbm.lbm_autotune(h, 2)
            tuned = True
        launch = lbm.lbm_get_launch(h)
        lbm.lbm_set_steps_per_pass(h, args.steps_per_pass, args.zplanes, args.tile_rows)
        spp, zplanes, tile_rows = lbm.lbm_get_steps_per_pass(h)
        placement = None
        if args.placement >= 2:
            tried, ms0, ms1 = lbm.lbm_tune_placement(h, args.placement, 1)
            placement = {"buffers_tried": tried, "ms_per_step_before": round(ms0, 4), "ms_per_step_after": round(ms1, 4)}

        lbm.lbm_step(h, args.warmup)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        lbm.lbm_step(h, args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev_ms = ev0.elapsed_time(ev1)
        mass, _ = lbm.lbm_totals(h)  # also checks the state is finite

        # Bandwidth probes on the same buffers: the pull-pattern copy (no
        # arithmetic, no boundary rule) and a plain contiguous copy.
        probes = {}
        for kind, name in ((1, "pull_pattern_copy"), (0, "read_write_copy")):
            lbm.lbm_probe(h, kind, 2)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lbm.lbm_probe(h, kind, args.probe_reps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.probe_reps
            # the pull-pattern copy moves the 19 N elements of the nodes, the
            # contiguous copy the whole buffer (in 16-byte units)
            moved = 19 * N * ebytes if kind == 1 else \
                lbm.lbm_buffer_elements(spec.nx, spec.ny, spec.nz, storage, layout) * ebytes // 16 * 16
            probes[name] = round(2 * moved / (ms * 1e-3) / 1e9, 1)
    finally:
        lbm.lbm_destroy(h)

    ms_per_step = wall * 1e3 / args.steps
    value = N * args.steps / wall / 1e6
    # launches in the timed region: one per step, or one per pair of steps
    # (an odd count ends with one single sweep)
    launches = args.steps // 2 + args.steps % 2 if spp == 2 else args.steps
    kernel_ms = ev_ms / launches
    alg_bytes = 2 * 19 * ebytes * N * args.steps / launches  # 19 loads + 19 stores per node update
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(launch, args.storage, args.layout, 2 if spp == 2 else 1,
                               [args.steps_per_pass, args.zplanes, args.tile_rows])
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {
            "workload": f"duct {spec.nx}x{spec.ny}x{spec.nz}, on-site Zou-He velocity inlet/outlet "
                        f"(0.04,0.01,0.01), on-site no-slip y/z walls, tau 0.8, {args.storage} storage",
            "nodes": N,
            "bytes_per_node_update": 2 * 19 * ebytes,
            "launch": {"block_x": launch[0], "nodes_per_thread": launch[1], "xcd_remap": launch[2],
                       "autotuned": tuned},
            "placement": placement,
            "layout": {"pop": "population-major", "rows": "row-major"}[args.layout],
            "steps_per_pass": spp,
            "z_planes": zplanes if spp == 2 else None,
            "tile_rows": (tile_rows or None) if spp == 2 else None,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": "sweep2_kernel" if spp == 2 else "sweep_kernel",
            "steps_per_launch": 2 if spp == 2 else 1,
            "kernel_ms_avg": round(kernel_ms, 4),
            # against the measured ceiling of the same access pattern: the pull-pattern
            # copy (streaming only) on the same buffers
            "frac_of_pull_copy": round(achieved / probes["pull_pattern_copy"], 4),
            # the best 50/50 read/write stream measured on the same buffers (a contiguous copy,
            # one 16-byte element per thread): the practical bandwidth ceiling of the device
            "ceiling_GBs": probes["read_write_copy"],
            "frac_of_ceiling": round(achieved / probes["read_write_copy"], 4),
            # the same kernel on the lattice's own two buffers, before placement tuning
            "frac_untuned_placement": None if placement is None else
            round(2 * 19 * ebytes * N / (placement["ms_per_step_before"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        },
        "probes_GBs": probes,
        "mass_after": mass,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds)
    legs = [x for x in args.legs.split(",") if x]
    if legs:
        out["forms"] = run_legs(args, legs)
    print(json.dumps(out), flush=True)


def run_legs(args, legs):
    """The systems forms beside the roofline run, each with its configured
    size (independent of --steps): the storage-precision gate on the
    512x256x256 duct (20000 steps), the 64-duct batch (2000 steps each) and a
    bounded serving trace.  A leg that fails reports its error instead of
    ending the run."""
    import torch

    forms = {}
    for leg in legs:
        t0 = time.perf_counter()
        try:
            if leg == "precision":
                r = form_precision(args, args.precision_steps)
                res = r["results"]
                forms[leg] = {
                    "workload": r["workload"], "steps": r["steps"],
                    "MLUPS": {k: v["MLUPS"] for k, v in res.items()},
                    "rel_L2_u_vs_f64": {k: res[k]["rel_L2_u_vs_f64"] for k in ("f32", "f16dev", "f16sr")},
                    "gate": {"f32_le_1e-5": res["f32"]["rel_L2_u_vs_f64"] <= 1e-5,
                             "f16sr_le_1e-3": res["f16sr"]["rel_L2_u_vs_f64"] <= 1e-3,
                             "f16dev_le_1e-3": res["f16dev"]["rel_L2_u_vs_f64"] <= 1e-3},
                    "f16sr_over_f32_MLUPS": r["f16sr_over_f32_MLUPS"],
                    "f16_over_f32_MLUPS": r["f16_over_f32_MLUPS"]}
            elif leg == "batch":
                r = form_batch(args, args.batch_steps)
                forms[leg] = {k: r[k] for k in ("lattices", "nodes", "steps_each", "shape", "batched",
                                                 "sequential_plain", "speedup", "bitwise_equal_to_plain")}
                forms[leg]["batched"]["GBs"] = round(r["batched"]["MLUPS"] * 152 / 1e3, 1)
            elif leg == "serve":
                r = form_serve(args, args.serve_requests)
                forms[leg] = r
            else:
                forms[leg] = {"error": "unknown leg"}
        except Exception as e:  # reported, not fatal: the roofline line above stands on its own
            forms[leg] = {"error": f"{type(e).__name__}: {e}"}
        forms.setdefault(leg, {})["leg_seconds"] = round(time.perf_counter() - t0, 1)
        print(f"leg {leg} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    return forms


if __name__ == "__main__":
    main()
