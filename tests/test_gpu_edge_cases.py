"""Edge cases through the C ABI: degenerate lattices (a single node, every
node a boundary node, one-node periodic axes) against the oracle step by
step; the FP16 forms at the full 512 x 256 x 256 size in the launch shape
the bench uses (sampled nodes recomputed by the oracle); all 64 seeded ducts
of the batch workload in one batch, a sample of them bit-identical alone."""
import numpy as np
import pytest

from lattice_symmetry import C as PAPER_C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_0811_4593_amd import lbm, serving, workloads  # noqa: E402

W = np.array([2] * 6 + [1] * 12 + [12]) / 36.0


def say(msg):
    print(msg, flush=True)


Z = (0.0, 0.0, 0.0)
DEGENERATE = [
    workloads.LatticeSpec(1, 1, 1, 0.8, {}, name="single_node_periodic"),
    workloads.LatticeSpec(1, 2, 1, 0.7, {}, name="1x2x1_periodic"),
    workloads.LatticeSpec(3, 3, 3, 0.9, {0: (0.02, 0.01, 0.0), 1: Z, 2: Z, 3: (0.0, 0.01, 0.02), 4: Z, 5: Z},
                          name="3x3x3_all_boundary"),
    workloads.LatticeSpec(1, 5, 4, 1.1, {2: Z, 3: (0.03, 0.0, 0.01), 4: Z, 5: Z}, name="1x5x4_x_single_periodic"),
    workloads.LatticeSpec(4, 1, 3, 0.75, {0: (0.01, 0.0, 0.02), 1: (0.01, 0.0, 0.02), 4: Z, 5: Z},
                          name="4x1x3_y_single_periodic"),
    workloads.LatticeSpec(3, 4, 1, 1.3, {0: Z, 1: Z, 2: (0.02, 0.0, 0.0), 3: Z}, name="3x4x1_z_single_periodic"),
]


@pytest.mark.parametrize("spec", DEGENERATE, ids=lambda s: s.name)
def test_degenerate_lattices_per_step_fp64(spec):
    L = oracle.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, bc=spec.bc)
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, 1.0, None, lbm.LBM_STORE_F64,
                       torch.cuda.current_stream())
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        lbm.lbm_set_populations(h, L.init(1.0, (0.01, -0.01, 0.02)) * workloads.perturbation(L.shape, 2, 0.05))
        cur, nxt = np.empty(L.shape), np.empty(L.shape)
        worst = 0.0
        for _ in range(10):
            lbm.lbm_get_populations(h, cur)
            expect = L.step(cur)
            lbm.lbm_step(h, 1)
            lbm.lbm_get_populations(h, nxt)
            worst = max(worst, float(np.max(np.abs(nxt - expect) / np.abs(expect))))
        say(f"{spec.name}: worst rel diff {worst:.2e}")
        assert worst <= 1e-12
    finally:
        lbm.lbm_destroy(h)


def _half_gap(x):
    ax = np.maximum(np.abs(x), 2.0 ** -14)
    return 2.0 ** (np.floor(np.log2(ax)) - 10)


def _sample(spec, rng, count=600):
    nx, ny, nz = spec.nx, spec.ny, spec.nz
    pts = [(rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)) for _ in range(count)]
    for x in (0, nx - 1):  # face, edge and corner nodes
        for y in (0, ny - 1, int(rng.integers(1, ny - 1))):
            for z in (0, nz - 1, int(rng.integers(1, nz - 1))):
                pts.append((x, y, z))
    pts += [(int(rng.integers(1, nx - 1)), y, int(rng.integers(0, nz))) for y in (0, ny - 1) for _ in range(20)]
    return np.array(pts, dtype=np.int64)


@pytest.mark.parametrize("storage,max_gaps", [(lbm.LBM_STORE_F16_DEV, 0.5), (lbm.LBM_STORE_F16_DEV_SR, 1.0)])
def test_full_size_precision_duct_fp16_sampled(storage, max_gaps):
    """512 x 256 x 256 duct, FP16 form, in the configuration the precision
    form times (row-major layout, launch shape from lbm_autotune, buffers
    from lbm_tune_placement): one step after those trial steps from rest;
    sampled
    nodes are recomputed by the oracle from the decoded FP16 state; the new
    scaled deviations must be within max_gaps of the half grid of the
    oracle's."""
    spec = workloads.precision_duct()
    nx, ny, nz = spec.nx, spec.ny, spec.nz
    stream = torch.cuda.current_stream()
    h = lbm.lbm_create(nx, ny, nz, spec.tau, 1.0, None, storage, stream)
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        lbm.lbm_set_layout(h, lbm.LBM_LAYOUT_ROW_MAJOR)
        lbm.lbm_step(h, 4)
        shape = lbm.lbm_autotune(h, 2)
        tried, _, _ = lbm.lbm_tune_placement(h, 3, 1)
        say(f"storage {storage}: row-major, autotuned {shape}, placement over {tried} buffers")
        host = np.empty((19, nz, ny, nx))
        lbm.lbm_get_populations(h, host)  # f = w + h 2^-8, exact decode
        pts = _sample(spec, np.random.default_rng(21))
        pulled = np.empty((len(pts), 19))
        for k in range(19):
            cxk, cyk, czk = (int(v) for v in PAPER_C[k])
            xs, ys, zs = pts[:, 0] - cxk, pts[:, 1] - cyk, pts[:, 2] - czk
            out = (xs < 0) | (xs >= nx) | (ys < 0) | (ys >= ny) | (zs < 0) | (zs >= nz)
            pulled[:, k] = np.where(out, np.nan, host[k, zs % nz, ys % ny, xs % nx])
        L = oracle.Lattice(nx, ny, nz, spec.tau, bc=spec.bc)
        expect = np.stack([L.update_node(int(a), int(b), int(c), p) for (a, b, c), p in zip(pts, pulled)])
        lbm.lbm_step(h, 1)
        lbm.lbm_get_populations(h, host)
        got = np.stack([host[:, c, b, a] for a, b, c in pts])
    finally:
        lbm.lbm_destroy(h)
    x = (expect - W[None, :]) * 256.0
    hv = (got - W[None, :]) * 256.0
    gap = _half_gap(x)
    err = np.abs(hv - x) - (max_gaps * gap + 256 * 1e-7)
    say(f"storage {storage}: {len(pts)} sampled nodes, worst excess over the bound {err.max():.2e}")
    assert np.all(err <= 0)


def test_batch_workload_64_ducts_sample_alone():
    specs = workloads.batch_ducts(64, seed=0)
    steps = 20
    run = serving.run_batch(specs, "f32", steps=steps, chunk=10, autotune=False, keep_results=True)
    assert all(s == steps for s in run.steps.values())
    rng = np.random.default_rng(7)
    for i in rng.choice(64, 6, replace=False):
        _, rho_p, u_p = serving.run_plain(specs[i], "f32", steps)
        np.testing.assert_array_equal(run.results[i][0], rho_p)
        np.testing.assert_array_equal(run.results[i][1], u_p)
    say(f"64 ducts ({sum(s.nodes for s in specs)} nodes), {steps} steps: sampled lattices bit-identical alone")
