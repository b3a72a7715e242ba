"""Pins of the oracle's pressure (density) boundary condition: the face rule
with the normal velocity computed from a prescribed density (Sec. IV eq_rhoin;
Appendix eq_voutx, eq_uinx, eq_uiny, eq_uouty and the top-plane form), the
edge closure eq_buried_rho and the corner closure of Sec. V, and the
square-channel experiment of Sec. VI (eq:squarechannel).

What the paper fixes, independently of the oracle's code:
  * a pressure face imposes the density exactly and keeps the prescribed
    tangential velocity; the unknowns follow from the same Ansatz as for a
    velocity face, so the result equals the velocity rule at the velocity the
    density implies;
  * equilibrium in gives equilibrium out;
  * on the edges and corners of a pressure plane the node's density becomes
    rho0 and its velocity stays zero; populations at rest with density rho0
    are a fixed point;
  * a pressure-driven flow between on-site no-slip plates is the parabola of
    eq_poiseuille with the gradient of the two prescribed densities, up to
    the compressibility of the lattice gas (second order in the density
    difference);
  * flow through a square channel converges to the series solution of
    eq:squarechannel with second order in the lattice spacing (Sec. VI: slope
    about 2).
"""
import itertools

import numpy as np
import pytest

from lattice_symmetry import C, NORMALS, cube_symmetries, face_of_normal, population_perm

W = np.array([2] * 6 + [1] * 12 + [12]) / 36.0
EDGES = [(a, b) for a, b in itertools.combinations(range(6), 2) if a // 2 != b // 2]
CORNERS = [(a, b, c) for a in (0, 1) for b in (2, 3) for c in (4, 5)]
WALL = (0.0, 0.0, 0.0)


def _unknown(faces):
    m = np.zeros(19, bool)
    for fc in faces:
        m |= C @ NORMALS[fc] > 0
    return m


def _tangential(face, v):
    n = NORMALS[face]
    v = np.asarray(v, float)
    return v - (v @ n) * n


# --------------------------------------------------------------------------
# Face rule
# --------------------------------------------------------------------------
@pytest.mark.parametrize("face", range(6))
@pytest.mark.parametrize("seed", range(4))
def test_pressure_face_imposes_density_and_tangential_velocity(oracle_mod, face, seed):
    rng = np.random.default_rng(40 * face + seed)
    f = rng.uniform(0.02, 0.12, 19)
    rho0 = rng.uniform(0.9, 1.2)
    v = rng.uniform(-0.05, 0.05, 3)  # its normal component must be ignored
    f_in = f.copy()
    f_in[_unknown([face])] = np.nan  # unknowns are never read
    g = oracle_mod.face_rule_pressure(face, rho0, v, f_in)
    assert np.isfinite(g).all()
    assert abs(g.sum() - rho0) <= 2e-16 * 19
    u = g @ C / g.sum()
    np.testing.assert_allclose(_tangential(face, u), _tangential(face, v), rtol=0, atol=3e-16)
    known = ~_unknown([face])
    np.testing.assert_array_equal(g[known], f[known])
    # The same closure as the velocity face: the velocity rule at the velocity
    # the density implies returns the same populations.
    g_vel = oracle_mod.face_rule(face, u, f)
    np.testing.assert_allclose(g_vel, g, rtol=0, atol=1e-15)


@pytest.mark.parametrize("face", range(6))
def test_pressure_face_equilibrium_is_a_fixed_point(oracle_mod, face):
    rho0 = 1.07
    u = np.array([0.03, -0.02, 0.025])
    feq = oracle_mod.feq(rho0, u)
    f = feq.copy()
    f[_unknown([face])] = np.nan
    # the tangential part of u is prescribed; the normal part must come out
    g = oracle_mod.face_rule_pressure(face, rho0, _tangential(face, u), f)
    np.testing.assert_allclose(g, feq, rtol=0, atol=4e-16)


def test_pressure_face_normal_component_ignored(oracle_mod):
    rng = np.random.default_rng(5)
    f = rng.uniform(0.02, 0.12, 19)
    a = oracle_mod.face_rule_pressure(4, 1.01, (0.01, 0.02, 0.0), f)
    b = oracle_mod.face_rule_pressure(4, 1.01, (0.01, 0.02, 0.37), f)
    np.testing.assert_array_equal(a, b)


def test_pressure_faces_are_symmetric_images(oracle_mod):
    rng = np.random.default_rng(9)
    f = rng.uniform(0.02, 0.12, 19)
    v = _tangential(4, rng.uniform(-0.05, 0.05, 3))
    g = oracle_mod.face_rule_pressure(4, 1.04, v, f)
    for R in cube_symmetries():
        p = population_perm(R)
        f2 = np.empty(19)
        f2[p] = f
        g2 = np.empty(19)
        g2[p] = g
        face2 = face_of_normal(R @ NORMALS[4])
        np.testing.assert_allclose(oracle_mod.face_rule_pressure(face2, 1.04, R @ v, f2), g2, rtol=0, atol=4e-16)


# --------------------------------------------------------------------------
# Edges and corners of a pressure plane
# --------------------------------------------------------------------------
@pytest.mark.parametrize("edge", EDGES)
def test_pressure_edge_density_velocity_and_buried(oracle_mod, edge):
    rng = np.random.default_rng(sum(edge))
    n1, n2 = NORMALS[edge[0]], NORMALS[edge[1]]
    buried = [int(np.flatnonzero((C == s * (n1 - n2)).all(axis=1))[0]) for s in (1, -1)]
    for _ in range(4):
        f = rng.uniform(0.02, 0.12, 19)
        rho0 = rng.uniform(0.9, 1.2)
        f_in = f.copy()
        f_in[_unknown(edge)] = np.nan
        g = oracle_mod.edge_rule_pressure(edge[0], edge[1], rho0, f_in)
        assert np.isfinite(g).all()
        assert abs(g.sum() - rho0) <= 4e-15
        np.testing.assert_allclose(g @ C, 0.0, atol=1e-16)
        # The buried pair shares one value and the rest population carries 12
        # times it; everything else is what the no-slip edge rule gives.
        assert g[buried[0]] == g[buried[1]]
        assert g[18] == 12.0 * g[buried[0]]
        g_ns = oracle_mod.edge_rule(edge[0], edge[1], f)
        others = np.ones(19, bool)
        others[buried + [18]] = False
        np.testing.assert_array_equal(g[others], g_ns[others])


@pytest.mark.parametrize("edge", EDGES)
def test_pressure_edge_rest_state_is_a_fixed_point(oracle_mod, edge):
    rho0 = 1.13
    f = W * rho0
    np.testing.assert_allclose(oracle_mod.edge_rule_pressure(edge[0], edge[1], rho0, f), f, rtol=1e-15)
    # a rest state of another density is brought to rho0
    g = oracle_mod.edge_rule_pressure(edge[0], edge[1], rho0, W * 0.97)
    assert abs(g.sum() - rho0) < 1e-15


@pytest.mark.parametrize("corner", CORNERS)
def test_pressure_corner_density_velocity_and_buried(oracle_mod, corner):
    rng = np.random.default_rng(sum(corner) + 50)
    s = NORMALS[corner[0]] + NORMALS[corner[1]] + NORMALS[corner[2]]
    buried = np.flatnonzero((C @ s == 0) & (np.arange(19) < 18))
    assert len(buried) == 6
    for _ in range(4):
        f = rng.uniform(0.02, 0.12, 19)
        rho0 = rng.uniform(0.9, 1.2)
        f_in = f.copy()
        f_in[_unknown(corner)] = np.nan
        g = oracle_mod.corner_rule_pressure(*corner, rho0, f_in)
        assert np.isfinite(g).all()
        assert abs(g.sum() - rho0) <= 4e-15
        np.testing.assert_allclose(g @ C, 0.0, atol=1e-16)
        assert np.all(g[buried] == g[buried[0]]) and g[18] == 12.0 * g[buried[0]]
        g_ns = oracle_mod.corner_rule(*corner, f)
        others = np.ones(19, bool)
        others[list(buried) + [18]] = False
        np.testing.assert_array_equal(g[others], g_ns[others])
    rho0 = 0.94
    np.testing.assert_allclose(oracle_mod.corner_rule_pressure(*corner, rho0, W * rho0), W * rho0, rtol=1e-15)


# --------------------------------------------------------------------------
# Lattices with pressure planes
# --------------------------------------------------------------------------
def test_pressure_lattice_validation(oracle_mod):
    f = np.ones((19, 5, 5, 5))
    with pytest.raises(ValueError):  # pressure planes on two axes meet at edges
        oracle_mod.Lattice(5, 5, 5, 0.8, bc={2: WALL, 3: WALL}, pressure={0: 1.0, 1: 1.0, 2: 1.0}).step(f)
    with pytest.raises(ValueError):  # non-positive density
        oracle_mod.Lattice(5, 5, 5, 0.8, bc={0: WALL, 1: WALL}, pressure={4: 0.0, 5: 1.0}).step(f)
    with pytest.raises(ValueError):  # one face of an axis only
        oracle_mod.Lattice(5, 5, 5, 0.8, pressure={4: 1.0}).step(f)
    # a pressure inlet with a velocity outlet on the same axis is allowed
    L = oracle_mod.Lattice(5, 5, 6, 0.8, bc={0: WALL, 1: WALL, 2: WALL, 3: WALL, 5: (0, 0, 0.01)},
                           pressure={4: 1.01})
    assert np.isfinite(L.step(L.init())).all()


def test_uniform_density_at_rest_is_a_fixed_point(oracle_mod):
    # Walls on x and y, both z planes at the same density as the fluid.
    rho0 = 1.02
    L = oracle_mod.Lattice(6, 5, 7, 0.9, bc={0: WALL, 1: WALL, 2: WALL, 3: WALL}, pressure={4: rho0, 5: rho0})
    f0 = L.init(rho0)
    f = L.run(f0, 40)
    np.testing.assert_allclose(f, f0, rtol=1e-14, atol=0)


def _transform(R, L, f):
    """Image of a lattice description (with pressure planes) and state under
    the cube symmetry R."""
    dims = np.array([L.nx, L.ny, L.nz])
    nd = np.abs(R) @ dims
    bc = {face_of_normal(R @ NORMALS[face]): tuple(R @ np.asarray(v, float)) for face, v in L.bc.items()}
    pr = {face_of_normal(R @ NORMALS[face]): r for face, r in L.pressure.items()}
    L2 = type(L)(int(nd[0]), int(nd[1]), int(nd[2]), L.tau, bc=bc, pressure=pr)
    z, y, x = np.meshgrid(np.arange(L.nz), np.arange(L.ny), np.arange(L.nx), indexing="ij")
    p2 = R @ np.stack([x, y, z]).reshape(3, -1)
    for a in range(3):
        if (R[a] < 0).any():
            p2[a] += nd[a] - 1
    g = np.empty((19, nd[2], nd[1], nd[0]))
    perm = population_perm(R)
    for k in range(19):
        g[perm[k], p2[2], p2[1], p2[0]] = f[k].reshape(-1)
    return L2, g


def test_cube_symmetry_of_a_pressure_duct_step(oracle_mod):
    rng = np.random.default_rng(21)
    L = oracle_mod.Lattice(6, 5, 7, 0.8, bc={0: WALL, 1: WALL, 2: WALL, 3: WALL, 4: (0.01, -0.02, 0.0)},
                           pressure={4: 1.02, 5: 0.99})
    f = L.init(1.0, (0.0, 0.0, 0.02)) * (1 + 0.05 * rng.uniform(-1, 1, L.shape))
    syms = cube_symmetries()
    for i in rng.choice(len(syms), 8, replace=False):
        R = syms[i]
        L2, g = _transform(R, L, f)
        _, expect = _transform(R, L, L.step(f))
        np.testing.assert_allclose(L2.step(g), expect, rtol=0, atol=1e-15)


def _steady(L, f, probe, check_every=200, rtol=1e-13, max_steps=40000):
    prev = None
    steps = 0
    while steps < max_steps:
        f = L.run(f, check_every)
        steps += check_every
        cur = probe(f)
        if prev is not None and np.abs(cur - prev).max() <= rtol * np.abs(cur).max():
            return f, steps
        prev = cur
    raise AssertionError("no steady state")


def _plane_poiseuille(oracle_mod, drho, tau):
    # No-slip plates at x = 0 and x = 15 (wall on the node: half width 7.5),
    # y periodic, pressure planes at z = 0 and z = 16 (edges of the pressure
    # planes with the plates use eq_buried_rho).
    nx, nz = 16, 17
    L = oracle_mod.Lattice(nx, 3, nz, tau, bc={0: WALL, 1: WALL}, pressure={4: 1 + drho / 2, 5: 1 - drho / 2})
    zm = (nz - 1) // 2

    def probe(f):
        return L.moments(f)[1][2, zm, 0]

    f, _ = _steady(L, L.init(), probe)
    rho, u = L.moments(f)
    grad = drho / 3.0 / (nz - 1)  # -dp/dz with p = rho / 3 (Sec. II)
    eta = (tau - 0.5) / 3.0 * rho[zm].mean()  # eq_visc
    x = np.arange(nx) - (nx - 1) / 2.0
    expect = grad / (2 * eta) * ((nx - 1) ** 2 / 4.0 - x ** 2)
    got = u[2, zm, 0]
    return np.abs(got - expect).max() / expect.max(), got, u


@pytest.mark.parametrize("tau", [1.0, 0.7])
def test_pressure_driven_plates_match_the_parabola(oracle_mod, tau):
    e_small, got, u = _plane_poiseuille(oracle_mod, 1e-4, tau)
    e_large, _, _ = _plane_poiseuille(oracle_mod, 1e-3, tau)
    # exact but for the compressibility: the error is second order in the
    # density difference (a mistake in the rule leaves a first-order or O(1) error)
    assert e_small < 2e-6
    assert 70 < e_large / e_small < 130
    assert max(abs(got[0]), abs(got[-1])) < 1e-16  # no slip on the plates, to rounding
    np.testing.assert_allclose(u[:2], 0.0, atol=1e-12)


def _square_channel_series(n, grad, eta, nterms=50):
    # eq:squarechannel with the wall on the boundary nodes: b = n - 1, origin
    # at the channel centre; returns v[y, x].
    b = n - 1.0
    c = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(c, c, indexing="xy")
    C_ = np.zeros_like(X)
    for k in range(nterms):
        q = (2 * k + 1) * np.pi / b
        C_ += (-1) ** k * np.cosh(q * X) * np.cos(q * Y) / ((2 * k + 1) ** 3 * np.cosh((2 * k + 1) * np.pi / 2))
    C_ *= 8 * b * b / np.pi ** 3
    return grad / (2 * eta) * (b * b / 4 - Y ** 2 - C_)


def _square_channel_error(oracle_mod, n, tau=1.0, umax=1e-3):
    nz = n + 1
    eta0 = (tau - 0.5) / 3.0
    grad = umax * 4 * eta0 / (0.2947 * (n - 1) ** 2)  # centre velocity ~ umax
    drho = 3.0 * grad * (nz - 1)
    L = oracle_mod.Lattice(n, n, nz, tau, bc={0: WALL, 1: WALL, 2: WALL, 3: WALL},
                           pressure={4: 1 + drho / 2, 5: 1 - drho / 2})
    zm = (nz - 1) // 2

    def probe(f):
        return L.moments(f)[1][2, zm]

    f, _ = _steady(L, L.init(), probe, rtol=1e-11)
    rho, u = L.moments(f)
    expect = _square_channel_series(n, drho / 3.0 / (nz - 1), eta0 * rho[zm].mean())
    return np.abs(u[2, zm] - expect).mean() / expect.max()


@pytest.mark.slow
def test_square_channel_second_order(oracle_mod):
    # Sec. VI: pressure in- and outlet (eq_rhoin), no-slip walls and edges;
    # mean relative error against the 50-term series for lattices 8..24 wide.
    ns = np.array([8, 12, 16, 24])
    errs = np.array([_square_channel_error(oracle_mod, int(n)) for n in ns])
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert 1.75 < slope < 2.25, (slope, errs)
    assert np.all(np.diff(errs) < 0)
    assert errs[-1] < 1e-3
