"""Pins of the oracle's whole time step (streaming, boundary rules, BGK)
against what the paper and the mathematics fix:

  * Couette flow between on-site walls (Sec. VI shear test): exact wall
    velocities at every step, the start-up transient of the diffusion equation
    with walls on the nodes, and a linear profile to rounding at steady state;
  * body-force Poiseuille flow between no-slip walls (Sec. VI, eq_gravity,
    eq_poiseuille, eq_visc) at tau = 1 and tau = 2: the parabola with no fit
    parameter, exactly zero velocity on the wall nodes;
  * invariants: mass and momentum conservation on periodic lattices, uniform
    flow stays uniform, translation and cube-symmetry equivariance of a whole
    step, exact prescribed velocities on every boundary node of a duct, and
    no unknown population ever read.
"""
import numpy as np
import pytest

from lattice_symmetry import NORMALS, cube_symmetries, face_of_normal, population_perm


def _near_eq_state(L, rng, amp=0.02):
    f = L.init(1.0, (0.01, -0.02, 0.015))
    return f * (1.0 + amp * rng.uniform(-1, 1, f.shape))


# --------------------------------------------------------------------------
# Couette
# --------------------------------------------------------------------------
def _couette_series(z, H, U, nu, t, nterms=4000):
    # u_t = nu u_zz, u(0) = 0, u(H) = U, u(z, 0) = 0.
    n = np.arange(1, nterms + 1)[:, None]
    return U * z / H + (2 * U / np.pi) * np.sum(
        ((-1.0) ** n / n) * np.sin(n * np.pi * z / H) * np.exp(-nu * (n * np.pi / H) ** 2 * t), axis=0)


def test_couette_startup_and_walls(oracle_mod):
    # x, y periodic; no-slip at z = 0, wall velocity (0.05, 0, 0) at z = 31,
    # tau = 1 (a narrow cross-section of the 16x16x32 configuration: the flow
    # is one-dimensional, so the cross-section does not matter).
    U, tau, nz = 0.05, 1.0, 32
    L = oracle_mod.Lattice(2, 2, nz, tau, bc={4: (0, 0, 0), 5: (U, 0, 0)})
    f = L.init()
    m0, _ = L.totals(f)
    for step in range(1, 2001):
        f = L.step(f)
        if step % 100 == 0 or step < 5:
            rho, u = L.moments(f)
            np.testing.assert_allclose(u[:, 0], 0.0, atol=1e-16)
            np.testing.assert_allclose(u[0, -1], U, rtol=0, atol=2e-16)
            np.testing.assert_allclose(u[1:, -1], 0.0, atol=1e-16)
    rho, u = L.moments(f)
    z = np.arange(nz, dtype=float)
    nu = (tau - 0.5) / 3.0
    series = _couette_series(z, nz - 1, U, nu, 2000)
    ux = u[0, :, 0, 0]
    # Not yet steady: the linear profile is still ~1e-3 away ...
    assert np.abs(ux - U * z / (nz - 1)).max() > 5e-4
    # ... but the start-up solution is met to 0.5% of that transient.
    assert np.abs(ux - series).max() < 5e-6
    # Wall-parallel flow: mass is conserved to rounding.
    m1, _ = L.totals(f)
    assert abs(m1 - m0) / m0 < 1e-13


@pytest.mark.slow
def test_couette_linear_at_steady_state(oracle_mod):
    U, nz = 0.05, 32
    L = oracle_mod.Lattice(2, 2, nz, 1.0, bc={4: (0, 0, 0), 5: (U, 0, 0)})
    f = L.run(L.init(), 20000)
    _, u = L.moments(f)
    z = np.arange(nz, dtype=float)
    # "linear flow profile within floating point precision" (Sec. VI)
    assert np.abs(u[0, :, 0, 0] - U * z / (nz - 1)).max() < 1e-13
    assert np.abs(u[1:]).max() < 1e-15


def test_couette_opposite_walls_paper_setup(oracle_mod):
    # The paper's shear test: v_x = +-0.02 on the two planes (32^3 there;
    # a 1x1x32 column here since x and y are periodic).
    L = oracle_mod.Lattice(1, 1, 32, 1.0, bc={4: (-0.02, 0, 0), 5: (0.02, 0, 0)})
    f = L.run(L.init(), 20000)
    _, u = L.moments(f)
    z = np.arange(32.0)
    assert np.abs(u[0, :, 0, 0] - (-0.02 + 0.04 * z / 31)).max() < 1e-14


# --------------------------------------------------------------------------
# Body-force Poiseuille
# --------------------------------------------------------------------------
@pytest.mark.parametrize("tau,steps", [(1.0, 16000), (2.0, 6000)])
def test_force_poiseuille(oracle_mod, tau, steps):
    # No-slip on-site walls at x = 0 and x = 31, y and z periodic, force along z.
    # Wall on the nodes: half width Delta x = 15.5 (Sec. V, wall position).
    F = 1e-6
    L = oracle_mod.Lattice(32, 4, 4, tau, bc={0: (0, 0, 0), 1: (0, 0, 0)}, force=(0, 0, F))
    f = L.init()
    for _ in range(steps):
        f = L.step(f)
    f, u_pre = L.step(f, want_u_pre=True)
    x = np.arange(32.0)
    eta = (tau - 0.5) / 3.0  # eq_visc with rho = 1
    expect = F / (2 * eta) * (15.5 ** 2 - (x - 15.5) ** 2)
    got = u_pre[2, 0, 0, :]
    assert np.abs(got - expect).max() / expect.max() < 1e-9
    assert got[0] == 0.0 and got[-1] == 0.0
    np.testing.assert_allclose(u_pre[:2], 0.0, atol=2e-15)


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------
def test_periodic_conservation(oracle_mod):
    rng = np.random.default_rng(1)
    L = oracle_mod.Lattice(7, 6, 5, 0.8)
    f = _near_eq_state(L, rng, 0.2)
    m0, j0 = L.totals(f)
    f = L.run(f, 10)
    m1, j1 = L.totals(f)
    assert abs(m1 - m0) / m0 < 1e-14
    np.testing.assert_allclose(j1, j0, rtol=0, atol=1e-14 * m0)


def test_uniform_flow_stays_uniform(oracle_mod):
    L = oracle_mod.Lattice(5, 4, 3, 0.7)
    u0 = (0.03, -0.02, 0.01)
    f0 = L.init(1.1, u0)
    f = L.run(f0, 7)
    np.testing.assert_allclose(f, f0, rtol=0, atol=1e-16)


def test_translation_equivariance(oracle_mod):
    rng = np.random.default_rng(2)
    L = oracle_mod.Lattice(6, 5, 4, 0.9)
    f = _near_eq_state(L, rng, 0.1)
    shift = (1, 2, 3)  # (z, y, x)
    a = np.roll(L.step(f), shift, axis=(1, 2, 3))
    b = L.step(np.roll(f, shift, axis=(1, 2, 3)))
    np.testing.assert_array_equal(a, b)


def _transform(R, L, f):
    """Image of a lattice description and state under the cube symmetry R."""
    dims = np.array([L.nx, L.ny, L.nz])
    nd = np.abs(R) @ dims
    bc = {}
    for face, v in L.bc.items():
        bc[face_of_normal(R @ NORMALS[face])] = tuple(R @ np.asarray(v, float))
    L2 = type(L)(int(nd[0]), int(nd[1]), int(nd[2]), L.tau, bc=bc, force=tuple(R @ np.asarray(L.force)))
    z, y, x = np.meshgrid(np.arange(L.nz), np.arange(L.ny), np.arange(L.nx), indexing="ij")
    pos = np.stack([x, y, z]).reshape(3, -1)
    p2 = R @ pos
    for a in range(3):
        if (R[a] < 0).any():
            p2[a] += nd[a] - 1
    g = np.empty((19, nd[2], nd[1], nd[0]))
    perm = population_perm(R)
    for k in range(19):
        g[perm[k], p2[2], p2[1], p2[0]] = f[k].reshape(-1)
    return L2, g


@pytest.mark.parametrize("seed", range(3))
def test_cube_symmetry_of_a_duct_step(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    v_in = (0.04, 0.01, 0.01)
    L = oracle_mod.Lattice(7, 5, 6, 0.8, bc={0: v_in, 1: v_in, 2: (0, 0, 0), 3: (0, 0, 0),
                                              4: (0, 0, 0), 5: (0, 0, 0)})
    f = _near_eq_state(L, rng, 0.05)
    syms = cube_symmetries()
    for i in rng.choice(len(syms), 8, replace=False):
        R = syms[i]
        L2, g = _transform(R, L, f)
        _, expect = _transform(R, L, L.step(f))
        np.testing.assert_allclose(L2.step(g), expect, rtol=0, atol=1e-15)  # summation order only


def test_all_boundary_nodes_meet_prescribed_velocity(oracle_mod):
    # A duct with all node classes: velocity faces at x, no-slip at y and z.
    # Moments of the stored (post-collision) state equal the post-boundary
    # ones (BGK conserves rho and rho u), so every face node reports its
    # prescribed velocity and every edge and corner node reports zero.
    v_in = np.array([0.04, 0.01, 0.01])
    L = oracle_mod.Lattice(9, 6, 5, 0.8, bc={0: v_in, 1: v_in, 2: (0, 0, 0), 3: (0, 0, 0),
                                             4: (0, 0, 0), 5: (0, 0, 0)})
    f = L.run(L.init(), 30)
    assert np.isfinite(f).all()
    _, u = L.moments(f)
    inner_yz = (slice(1, -1), slice(1, -1))
    for xs in (0, -1):
        np.testing.assert_allclose(u[:, inner_yz[0], inner_yz[1], xs].reshape(3, -1).T, np.broadcast_to(v_in, (12, 3)),
                                   rtol=0, atol=1e-16)
    for sl in [(slice(None), 0, slice(None), slice(1, -1)), (slice(None), -1, slice(None), slice(1, -1)),
               (slice(None), slice(None), 0, slice(1, -1)), (slice(None), slice(None), -1, slice(1, -1))]:
        np.testing.assert_allclose(u[sl], 0.0, atol=1e-16)
    # edges and corners on the velocity planes are no-slip as well
    for xs in (0, -1):
        for zs in (0, -1):
            np.testing.assert_allclose(u[:, zs, :, xs], 0.0, atol=1e-16)
        for ys in (0, -1):
            np.testing.assert_allclose(u[:, :, ys, xs], 0.0, atol=1e-16)


def test_invalid_lattices_are_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.Lattice(5, 5, 5, 0.5).step(np.ones((19, 5, 5, 5)))
    with pytest.raises(ValueError):  # one face of an axis only
        oracle_mod.Lattice(5, 5, 5, 0.8, bc={4: (0, 0, 0)}).step(np.ones((19, 5, 5, 5)))
    with pytest.raises(ValueError):  # bounded axis shorter than 3 nodes
        oracle_mod.Lattice(5, 5, 2, 0.8, bc={4: (0, 0, 0), 5: (0, 0, 0)}).step(np.ones((19, 2, 5, 5)))


def test_thread_count_does_not_change_results(oracle_mod):
    rng = np.random.default_rng(4)
    L = oracle_mod.Lattice(8, 7, 9, 0.8, bc={0: (0.04, 0.01, 0.01), 1: (0.04, 0.01, 0.01),
                                             2: (0, 0, 0), 3: (0, 0, 0), 4: (0, 0, 0), 5: (0, 0, 0)})
    f = _near_eq_state(L, rng)
    np.testing.assert_array_equal(L.step(f, nthreads=1), L.step(f, nthreads=4))
