"""The wall comparisons of Sec. VI on the GPU (FP64 storage).

* Body-force Poiseuille (eq_gravity paragraph): the rule keeps the wall
  nodes at zero velocity at tau = 1 and 2; simple bounce-back (the rule
  without the corrections N, lbm_set_rule_options) slips by 2 tau F / rho,
  the closed form derived in test_oracle_wall_comparisons.py, and the
  profile is the parabola lifted by that slip.
* Square channel (eq:squarechannel paragraph): per-step parity with the
  oracle for the bounce-back channel (solid boundary nodes, pressure in- and
  outlet), then the convergence study over 8..48 nodes: the rule second
  order; bounce-back with the wall taken on the boundary nodes first order;
  with the wall half a spacing inside (mid-grid) second order; the rule's
  error the smallest at every size.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_0811_4593_amd import lbm, workloads  # noqa: E402

WALL = (0.0, 0.0, 0.0)


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("tau,steps", [(1.0, 16000), (2.0, 6000)])
def test_force_poiseuille_slip_without_corrections_on_gpu(tau, steps):
    nx, ny, nz, F = 32, 4, 4, 1e-6
    x = np.arange(nx, dtype=float)
    expect = F / (2 * (tau - 0.5) / 3.0) * (15.5 ** 2 - (x - 15.5) ** 2)
    for no_n in (False, True):
        h = lbm.lbm_create(nx, ny, nz, tau, 1.0, None, lbm.LBM_STORE_F64, torch.cuda.current_stream())
        try:
            lbm.lbm_set_velocity_bc(h, 0, WALL)
            lbm.lbm_set_velocity_bc(h, 1, WALL)
            lbm.lbm_set_body_force(h, (0.0, 0.0, F))
            if no_n:
                lbm.lbm_set_rule_options(h, lbm.LBM_RULE_NO_TRANSVERSE)
            lbm.lbm_step(h, steps)
            rho, u = np.empty(nx * ny * nz), np.empty(3 * nx * ny * nz)
            lbm.lbm_moments(h, rho, u)
        finally:
            lbm.lbm_destroy(h)
        rho = rho.reshape(nz, ny, nx)[0, 0]
        # the stored state carries rho u + F; the post-boundary velocity is (j - F) / rho
        uz = (u.reshape(3, nz, ny, nx)[2, 0, 0] * rho - F) / rho
        if no_n:
            slip = 2 * tau * F / rho[0]
            say(f"tau {tau}: wall velocity without N {uz[0]:.6e} (2 tau F / rho = {slip:.6e})")
            np.testing.assert_allclose(uz[[0, -1]], slip, rtol=1e-8)
            assert np.abs(uz - (expect + slip)).max() / expect.max() < 1e-8
        else:
            assert np.abs(uz[[0, -1]]).max() < 1e-15
            assert np.abs(uz - expect).max() / expect.max() < 1e-9


def _bounce_back_channel(n, tau, drho):
    nz = n + 1
    solid = np.zeros((nz, n, n), np.uint8)
    solid[:, 0, :] = solid[:, -1, :] = solid[:, :, 0] = solid[:, :, -1] = 1
    return solid, {4: 1 + drho / 2, 5: 1 - drho / 2}


def test_bounce_back_square_channel_per_step_parity():
    n, tau = 12, 0.9
    solid, pressure = _bounce_back_channel(n, tau, 2e-3)
    nz = n + 1
    L = oracle.Lattice(n, n, nz, tau, pressure=pressure, solid=solid)
    h = lbm.lbm_create(n, n, nz, tau, 1.0, None, lbm.LBM_STORE_F64, torch.cuda.current_stream())
    try:
        for face, r in pressure.items():
            lbm.lbm_set_pressure_bc(h, face, r)
        lbm.lbm_set_solid_mask(h, solid)
        lbm.lbm_set_populations(h, L.init(1.0, (0.0, 0.0, 0.01)) * workloads.perturbation(L.shape, 4, 0.05))
        cur, nxt = np.empty(L.shape), np.empty(L.shape)
        worst = 0.0
        for _ in range(10):
            lbm.lbm_get_populations(h, cur)
            expect = L.step(cur)
            lbm.lbm_step(h, 1)
            lbm.lbm_get_populations(h, nxt)
            worst = max(worst, float(np.max(np.abs(nxt - expect) / np.abs(expect))))
        say(f"bounce-back square channel {n}: worst rel diff {worst:.2e}")
        assert worst <= 1e-12
    finally:
        lbm.lbm_destroy(h)


def _series(n, b, grad, eta, nterms=50):
    c = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(c, c, indexing="xy")
    acc = np.zeros_like(X)
    for k in range(nterms):
        q = (2 * k + 1) * np.pi / b
        acc += (-1) ** k * np.cosh(q * X) * np.cos(q * Y) / ((2 * k + 1) ** 3 * np.cosh((2 * k + 1) * np.pi / 2))
    acc *= 8 * b * b / np.pi ** 3
    return grad / (2 * eta) * (b * b / 4 - Y ** 2 - acc)


def _channel_errors(n, variant, tau=1.0, umax=1e-3, rtol=1e-11):
    nz = n + 1
    eta0 = (tau - 0.5) / 3.0
    grad = umax * 4 * eta0 / (0.2947 * (n - 1) ** 2)
    drho = 3.0 * grad * (nz - 1)
    solid, pressure = _bounce_back_channel(n, tau, drho)
    h = lbm.lbm_create(n, n, nz, tau, 1.0, None, lbm.LBM_STORE_F64, torch.cuda.current_stream())
    try:
        for face, r in pressure.items():
            lbm.lbm_set_pressure_bc(h, face, r)
        fluid = np.ones((n, n), bool)
        if variant == "bounce_back":
            lbm.lbm_set_solid_mask(h, solid)
            fluid = solid[0] == 0
            widths = {"b=n-1": n - 1.0, "b=n-2": n - 2.0}
        else:
            for face in range(4):
                lbm.lbm_set_velocity_bc(h, face, WALL)
            if variant == "no_n":
                lbm.lbm_set_rule_options(h, lbm.LBM_RULE_NO_TRANSVERSE)
            widths = {"b=n-1": n - 1.0}
        N = n * n * nz
        rho, u = np.empty(N), np.empty(3 * N)
        zm = (nz - 1) // 2
        prev, steps = None, 0
        while True:
            lbm.lbm_step(h, 200)
            steps += 200
            lbm.lbm_moments(h, rho, u)
            cur = u.reshape(3, nz, n, n)[2, zm].copy()
            if prev is not None and np.abs(cur - prev).max() <= rtol * np.abs(cur).max():
                break
            assert steps < 100000, "no steady state"
            prev = cur
    finally:
        lbm.lbm_destroy(h)
    g = drho / 3.0 / (nz - 1)
    eta = eta0 * rho.reshape(nz, n, n)[zm].mean()
    out = {}
    for name, b in widths.items():
        e = _series(n, b, g, eta)
        out[name] = float(np.abs(cur - e)[fluid].mean() / e[fluid].max())
    return out, steps


def _slope(ns, errs):
    return float(-np.polyfit(np.log(ns), np.log(errs), 1)[0])


def test_square_channel_rule_against_bounce_back_on_gpu():
    ns = np.array([8, 12, 16, 24, 32, 48])
    rule, node_bb, mid_bb, no_n = [], [], [], []
    for n in ns:
        r, s1 = _channel_errors(int(n), "rule")
        bb, s2 = _channel_errors(int(n), "bounce_back")
        nn, _ = _channel_errors(int(n), "no_n")
        rule.append(r["b=n-1"])
        node_bb.append(bb["b=n-1"])
        mid_bb.append(bb["b=n-2"])
        no_n.append(nn["b=n-1"])
        say(f"n {n}: rule {rule[-1]:.3e} ({s1} steps), node bounce-back {node_bb[-1]:.3e}, "
            f"mid-grid {mid_bb[-1]:.3e} ({s2} steps), without N {no_n[-1]:.3e}")
    rule, node_bb, mid_bb, no_n = map(np.array, (rule, node_bb, mid_bb, no_n))
    s_rule, s_node, s_mid, s_non = (_slope(ns, e) for e in (rule, node_bb, mid_bb, no_n))
    say(f"slopes: rule {s_rule:.2f}, node bounce-back {s_node:.2f}, mid-grid {s_mid:.2f}, without N {s_non:.2f}")
    assert 1.8 < s_rule < 2.2
    assert 0.9 < s_node < 1.5
    assert 1.8 < s_mid < 3.0
    assert np.all(rule < mid_bb) and np.all(mid_bb < node_bb)
    assert np.all(rule < no_n)
