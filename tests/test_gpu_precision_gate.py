"""Storage-precision gate at full size: the 512 x 256 x 256 duct (no-slip
on-site walls on the y and z faces, on-site velocity inlet and outlet
(0.04, 0.01, 0.01), tau 0.8) run for 20000 steps from rest in every storage
form, in the row-major layout and default launch shape the library starts
with.  The reference is the FP64 form, whose per-step parity with the CPU
oracle (1e-12) is pinned in test_gpu_parity.py.

Bars (relative L2 of the velocity field against FP64):
* FP32 storage (arithmetic in double): <= 1e-5;
* FP16 scaled deviations with stochastic rounding (arithmetic in FP32):
  <= 1e-3.
The FP16 form with round-to-nearest-even misses the 1e-3 bar on this run
(its rounding is the same at every step of a steady state and acts as a
constant forcing); its error is measured and printed, and held to its
documented value (< 2.5e-3) so that a regression still fails.
"""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0811_4593_amd import lbm, workloads  # noqa: E402

STEPS = 20000


def say(msg):
    print(msg, flush=True)


def run_form(storage):
    """Velocity field [3][N] (device, float64) of the duct after STEPS steps."""
    spec = workloads.precision_duct()
    stream = torch.cuda.current_stream()
    h = lbm.lbm_create(spec.nx, spec.ny, spec.nz, spec.tau, spec.rho0, None, storage, stream)
    try:
        for face, v in spec.bc.items():
            lbm.lbm_set_velocity_bc(h, face, v)
        assert lbm.lbm_get_layout(h) == lbm.LBM_LAYOUT_ROW_MAJOR
        for done in range(0, STEPS, 2000):
            lbm.lbm_step(h, 2000)
            torch.cuda.synchronize()
            if done % 10000 == 0:
                say(f"  {lbm.STORAGE_NAMES[storage]}: {done + 2000} steps")
        mass, _ = lbm.lbm_totals(h)  # raises if the state is not finite
        u = torch.empty(3 * spec.nodes, dtype=torch.float64, device="cuda")
        lbm.lbm_moments(h, None, u, dst_on_device=True)
        return u, mass
    finally:
        lbm.lbm_destroy(h)


@pytest.fixture(scope="module")
def u_f64():
    say("precision gate: FP64 reference, 512x256x256, 20000 steps")
    u, mass = run_form(lbm.LBM_STORE_F64)
    say(f"  FP64 mass {mass:.6e}")
    yield u
    del u
    torch.cuda.empty_cache()


def rel_l2(u, ref):
    return float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(ref))


def test_fp32_storage_within_1e5(u_f64):
    u, _ = run_form(lbm.LBM_STORE_F32)
    e = rel_l2(u, u_f64)
    say(f"FP32 storage: rel L2 u vs FP64 = {e:.3e}")
    assert e <= 1e-5


def test_fp16_stochastic_rounding_within_1e3(u_f64):
    u, _ = run_form(lbm.LBM_STORE_F16_DEV_SR)
    e = rel_l2(u, u_f64)
    say(f"FP16 SR storage: rel L2 u vs FP64 = {e:.3e}")
    assert e <= 1e-3


def test_fp16_round_to_nearest_measured(u_f64):
    u, _ = run_form(lbm.LBM_STORE_F16_DEV)
    e = rel_l2(u, u_f64)
    say(f"FP16 RNE storage: rel L2 u vs FP64 = {e:.3e} (documented: misses 1e-3 on this run)")
    assert e < 2.5e-3
