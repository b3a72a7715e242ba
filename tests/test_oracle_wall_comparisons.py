"""The wall comparisons of Sec. VI, on the oracle.

Body-force Poiseuille (the eq_gravity paragraph): with the paper's rule the
wall nodes carry exactly zero velocity at tau = 1 and tau = 2; with simple
bounce-back (the face rule without the transverse corrections N, v = 0) the
paper observes a numerical slip.  Its size follows in closed form: at a
wall node the bounced diagonals cancel the outgoing ones in the tangential
momentum, which is left with the in-plane populations; those stream within
the wall plane, so at steady state they relax onto themselves, and the
in-plane share (2/3) of the equilibrium momentum rho u + tau F (the body
force shifts the equilibrium velocity by tau F / rho) balances when
rho u_wall = 2 tau F.  The slip is therefore tau-dependent, 2 tau F / rho,
and the whole profile is the parabola lifted by it.

Square channel (eq:squarechannel paragraph and the caption of its figure):
the rule (wall on the boundary nodes, b = n - 1 spacings) converges with
second order.  Bounce-back at solid boundary nodes (populations streaming
in from a solid node return as the node's own opposite population) is
compared with the wall taken on the boundary nodes (node-based bounce-back,
b = n - 1: first order, the kink next to the wall) and with the wall half a
spacing inside (mid-grid bounce-back, b = n - 2: second order again).  The
rule without N (on-site bounce-back of the unknowns) is reported beside
them.  Every error is the mean absolute deviation over the fluid nodes of
the middle cross-section divided by the series' maximum there.
"""
import numpy as np
import pytest

WALL = (0.0, 0.0, 0.0)


def _poiseuille(oracle_mod, tau, steps, no_n, F=1e-6):
    L = oracle_mod.Lattice(32, 4, 4, tau, bc={0: WALL, 1: WALL}, force=(0, 0, F), no_transverse=no_n)
    f = L.run(L.init(), steps)
    f, u_pre = L.step(f, want_u_pre=True)
    rho, _ = L.moments(f)
    x = np.arange(32.0)
    expect = F / (2 * (tau - 0.5) / 3.0) * (15.5 ** 2 - (x - 15.5) ** 2)  # eq_poiseuille, eq_visc
    return u_pre[2, 0, 0, :], rho[0, 0, :], expect


@pytest.mark.parametrize("tau,steps", [(1.0, 16000), (2.0, 6000)])
def test_force_poiseuille_slip_without_corrections(oracle_mod, tau, steps):
    F = 1e-6
    got, _, expect = _poiseuille(oracle_mod, tau, steps, False, F)
    assert got[0] == 0.0 and got[-1] == 0.0  # the rule: no slip at all
    assert np.abs(got - expect).max() / expect.max() < 1e-9
    got_b, rho_b, _ = _poiseuille(oracle_mod, tau, steps, True, F)
    slip = 2 * tau * F / rho_b[0]
    np.testing.assert_allclose(got_b[[0, -1]], slip, rtol=1e-8)
    # the profile is the parabola lifted by the slip
    assert np.abs(got_b - (expect + slip)).max() / expect.max() < 1e-8


def _series(n, b, grad, eta, nterms=50):
    # eq:squarechannel, origin at the centre of the n x n cross-section, half
    # width b / 2; returns v[y, x]
    c = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(c, c, indexing="xy")
    acc = np.zeros_like(X)
    for k in range(nterms):
        q = (2 * k + 1) * np.pi / b
        acc += (-1) ** k * np.cosh(q * X) * np.cos(q * Y) / ((2 * k + 1) ** 3 * np.cosh((2 * k + 1) * np.pi / 2))
    acc *= 8 * b * b / np.pi ** 3
    return grad / (2 * eta) * (b * b / 4 - Y ** 2 - acc)


def _steady(L, f, probe, every=200, rtol=1e-11, max_steps=60000):
    prev, steps = None, 0
    while steps < max_steps:
        f = L.run(f, every)
        steps += every
        cur = probe(f)
        if prev is not None and np.abs(cur - prev).max() <= rtol * np.abs(cur).max():
            return f
        prev = cur
    raise AssertionError("no steady state")


def square_channel_errors(oracle_mod, n, variant, tau=1.0, umax=1e-3):
    """Mean relative error(s) of one square-channel variant: 'rule', 'no_n'
    ({'b=n-1': e}) or 'bounce_back' ({'b=n-1': node-based, 'b=n-2':
    mid-grid})."""
    nz = n + 1
    eta0 = (tau - 0.5) / 3.0
    grad = umax * 4 * eta0 / (0.2947 * (n - 1) ** 2)
    drho = 3.0 * grad * (nz - 1)
    pressure = {4: 1 + drho / 2, 5: 1 - drho / 2}
    fluid = np.ones((n, n), bool)
    if variant == "bounce_back":
        solid = np.zeros((nz, n, n), bool)
        solid[:, 0, :] = solid[:, -1, :] = solid[:, :, 0] = solid[:, :, -1] = True
        L = oracle_mod.Lattice(n, n, nz, tau, pressure=pressure, solid=solid)
        fluid = ~solid[0]
        widths = {"b=n-1": n - 1.0, "b=n-2": n - 2.0}
    else:
        L = oracle_mod.Lattice(n, n, nz, tau, bc={0: WALL, 1: WALL, 2: WALL, 3: WALL}, pressure=pressure,
                               no_transverse=variant == "no_n")
        widths = {"b=n-1": n - 1.0}
    zm = (nz - 1) // 2
    f = _steady(L, L.init(), lambda f: L.moments(f)[1][2, zm])
    rho, u = L.moments(f)
    g = drho / 3.0 / (nz - 1)
    eta = eta0 * rho[zm].mean()
    out = {}
    for name, b in widths.items():
        e = _series(n, b, g, eta)
        out[name] = float(np.abs(u[2, zm] - e)[fluid].mean() / e[fluid].max())
    return out


def slope(ns, errs):
    return float(-np.polyfit(np.log(ns), np.log(errs), 1)[0])


@pytest.mark.slow
def test_square_channel_rule_against_bounce_back(oracle_mod):
    ns = np.array([8, 12, 16, 24])
    rule = np.array([square_channel_errors(oracle_mod, int(n), "rule")["b=n-1"] for n in ns])
    bb = [square_channel_errors(oracle_mod, int(n), "bounce_back") for n in ns]
    node_bb = np.array([e["b=n-1"] for e in bb])
    mid_bb = np.array([e["b=n-2"] for e in bb])
    no_n = np.array([square_channel_errors(oracle_mod, int(n), "no_n")["b=n-1"] for n in ns])
    s_rule, s_node, s_mid = slope(ns, rule), slope(ns, node_bb), slope(ns, mid_bb)
    print(f"rule {rule} slope {s_rule:.2f}; node bounce-back {node_bb} slope {s_node:.2f}; "
          f"mid-grid {mid_bb} slope {s_mid:.2f}; without N {no_n} slope {slope(ns, no_n):.2f}")
    assert 1.75 < s_rule < 2.25
    assert 0.9 < s_node < 1.5          # first order: the wall is not where it is assumed
    assert 1.8 < s_mid < 3.0           # second order once the wall sits half-way
    assert np.all(rule < mid_bb) and np.all(mid_bb < node_bb)
    assert np.all(rule < no_n)
