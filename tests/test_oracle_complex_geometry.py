"""Pins of the oracle's complex-geometry wall nodes (Sec. V: per-node rule
from the geometry, convex edges eq_edge2, points where edges meet planes),
on random populations and small lattices.

What fixes them:
  * a box described as a geometry (walls on its boundary nodes, solid
    interior outside) is the box with on-site no-slip faces, edges and
    corners, node by node;
  * the convex-edge rule bounces back the one unknown population, leaves
    every population but the five it names alone, makes the momentum along
    the edge vanish and keeps a fluid at rest at rest;
  * the general rule keeps a fluid at rest at rest for any unknown set, gives
    the buried links and the rest population the others' mass in the ratio
    of their weights (eq_buried's 22 and eq_corner's 18 as special cases);
  * plane, concave-edge and corner nodes of a geometry meet zero velocity
    exactly; a step with a geometry commutes with the cube symmetries.
"""
import itertools

import numpy as np
import pytest

from lattice_symmetry import C, NORMALS, cube_symmetries, face_of_normal, population_perm

from paper_0811_4593_amd import workloads

W = np.array([2] * 6 + [1] * 12 + [12]) / 36.0
OPP = np.array([int(np.flatnonzero((C == -c).all(axis=1))[0]) for c in C])


def _box_geometry(a, b, c):
    """Node types of a box of a x b x c wall-and-fluid nodes inside one layer
    of solid interior (lattice (a+2) x (b+2) x (c+2))."""
    solid = np.ones((c + 2, b + 2, a + 2), bool)
    solid[2:c, 2:b, 2:a] = False
    return workloads.cells_from_solid(solid)


def test_box_as_geometry_is_the_coordinate_box(oracle_mod):
    a, b, c = 7, 6, 5
    cell = _box_geometry(a, b, c)
    assert (cell[1:-1, 1:-1, 1:-1] != 2).all() and (cell[1:-1, 1:-1, 1:-1] == 1).sum() == a * b * c - (a - 2) * (b - 2) * (c - 2)
    G = oracle_mod.Lattice(a + 2, b + 2, c + 2, 0.85, cell=cell)
    B = oracle_mod.Lattice(a, b, c, 0.85, bc={f: (0.0, 0.0, 0.0) for f in range(6)})
    rng = np.random.default_rng(4)
    fb = B.init(1.0, (0.01, -0.02, 0.015)) * (1 + 0.05 * rng.uniform(-1, 1, B.shape))
    fg = G.init()
    fg[:, 1:-1, 1:-1, 1:-1] = fb
    for _ in range(5):
        fb = B.step(fb)
        fg = G.step(fg)
        np.testing.assert_array_equal(fg[:, 1:-1, 1:-1, 1:-1], fb)


def test_classification_of_the_box(oracle_mod):
    cell = _box_geometry(6, 5, 4)
    L = oracle_mod.Lattice(8, 7, 6, 0.8, cell=cell)
    kinds = {}
    for z, y, x in zip(*np.nonzero(cell == 1)):
        k, _ = L.classify(x, y, z)
        kinds[k] = kinds.get(k, 0) + 1
    # 8 corners, 4 (a-2) + 4 (b-2) + 4 (c-2) edge nodes, the rest plane nodes
    assert kinds[oracle_mod.NODE_CORNER] == 8
    assert kinds[oracle_mod.NODE_EDGE] == 4 * (4 + 3 + 2)
    assert kinds[oracle_mod.NODE_FACE] == 2 * (4 * 3 + 4 * 2 + 3 * 2)
    assert set(kinds) == {oracle_mod.NODE_FACE, oracle_mod.NODE_EDGE, oracle_mod.NODE_CORNER}


CONVEX = [(a, b) for a, b in itertools.combinations(range(6), 2) if a // 2 != b // 2]


@pytest.mark.parametrize("edge", CONVEX)
def test_convex_edge_rule(oracle_mod, edge):
    n1, n2 = NORMALS[edge[0]], NORMALS[edge[1]]
    e = np.cross(n1, n2)
    i_in = int(np.flatnonzero((C == n1 + n2).all(axis=1))[0])
    corrected = [i for i in range(18) if C[i] @ e != 0 and C[i] @ (n1 + n2) == 1]
    assert len(corrected) == 4
    rng = np.random.default_rng(sum(edge))
    for _ in range(4):
        f = rng.uniform(0.02, 0.12, 19)
        f_in = f.copy()
        f_in[i_in] = np.nan
        g = oracle_mod.convex_edge_rule(edge[0], edge[1], f_in)
        assert np.isfinite(g).all()
        assert abs(g @ C @ e) < 1e-16                            # no momentum along the edge
        changed = np.flatnonzero(g != f)
        assert set(changed) <= set(corrected) | {i_in}
        h = f.copy()
        h[i_in] = f[OPP[i_in]]
        assert abs(g.sum() - h.sum()) < 1e-15                   # the correction moves no mass
    np.testing.assert_allclose(oracle_mod.convex_edge_rule(edge[0], edge[1], W * 1.1), W * 1.1, rtol=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_general_rule(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    unknown = rng.uniform(size=18) < 0.4
    mask = int(sum(1 << i for i in range(18) if unknown[i]))
    np.testing.assert_allclose(oracle_mod.general_rule(mask, W * 0.93), W * 0.93, rtol=1e-15)
    f = rng.uniform(0.02, 0.12, 19)
    f_in = f.copy()
    f_in[:18][unknown] = np.nan
    f_in[18] = np.nan  # the rest population is reassigned: never read
    g = oracle_mod.general_rule(mask, f_in)
    assert np.isfinite(g).all()
    buried = unknown & unknown[OPP[:18]]
    bounced = unknown & ~buried
    np.testing.assert_array_equal(g[:18][bounced], f[OPP[:18]][bounced])
    np.testing.assert_array_equal(g[:18][~unknown], f[:18][~unknown])
    nb = ~buried
    share = g[:18][nb].sum() / W[:18][nb].sum()
    np.testing.assert_allclose(g[:18][buried], W[:18][buried] * share, rtol=1e-14)
    assert abs(g[18] - W[18] * share) < 1e-15


def test_general_rule_reduces_to_edge_and_corner_closures(oracle_mod):
    f = np.random.default_rng(1).uniform(0.02, 0.12, 19)
    for edge in [(0, 2), (1, 4), (3, 5)]:
        U = (C @ NORMALS[edge[0]] > 0) | (C @ NORMALS[edge[1]] > 0)
        mask = int(sum(1 << i for i in range(18) if U[i]))
        g_gen = oracle_mod.general_rule(mask, f)
        g_edge = oracle_mod.edge_rule(edge[0], edge[1], f)
        # the same closure; the edge rule adds the correction along the edge
        e = np.cross(NORMALS[edge[0]], NORMALS[edge[1]])
        same = np.array([C[i] @ e == 0 for i in range(19)])
        np.testing.assert_allclose(g_gen[same], g_edge[same], rtol=1e-14)


def _random_blocks(seed, shape=(10, 11, 12), count=3):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    solid = np.zeros(shape, bool)
    for _ in range(count):  # blocks at least 3 nodes thick have an interior
        x0, y0, z0 = rng.integers(0, [nx - 5, ny - 5, nz - 5])
        w = rng.integers(3, 6, 3)
        solid[z0:z0 + w[2], y0:y0 + w[1], x0:x0 + w[0]] = True
    return workloads.cells_from_solid(solid)


def _rib(oracle_mod, force=(0.0, 0.0, 0.0)):
    spec, cell = workloads.rib_channel()
    return oracle_mod.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, force=force, cell=cell), cell


def test_rib_channel_node_kinds(oracle_mod):
    L, cell = _rib(oracle_mod)
    kinds = {}
    for z, y, x in zip(*np.nonzero(cell == 1)):
        k, _ = L.classify(x, y, z)
        kinds[k] = kinds.get(k, 0) + 1
    # two convex edges along y across the 6 fluid rows (y = 2..7)
    assert kinds[oracle_mod.NODE_CONVEX_EDGE] == 2 * 6
    assert kinds[oracle_mod.NODE_GENERAL] > 0 and kinds[oracle_mod.NODE_EDGE] > 0


def test_rib_channel_walls_at_rest_and_convex_edges(oracle_mod):
    L, cell = _rib(oracle_mod)
    rng = np.random.default_rng(6)
    f = L.init(1.0, (0.02, 0.0, 0.0)) * (1 + 0.02 * rng.uniform(-1, 1, L.shape))
    f = L.step(f)
    _, u = L.moments(f)  # no force: post-collision moments = post-rule moments
    for z, y, x in zip(*np.nonzero(cell == 1)):
        k, _ = L.classify(x, y, z)
        if k in (oracle_mod.NODE_FACE, oracle_mod.NODE_EDGE, oracle_mod.NODE_CORNER):
            assert np.abs(u[:, z, y, x]).max() < 1e-16
        elif k == oracle_mod.NODE_CONVEX_EDGE:
            assert abs(u[1, z, y, x]) < 1e-16  # the edges run along y
    # a fluid at rest stays at rest
    f0 = L.init(1.03)
    np.testing.assert_allclose(L.run(f0, 10)[:, cell != 2], f0[:, cell != 2], rtol=1e-14)


def test_geometry_step_commutes_with_cube_symmetries(oracle_mod):
    rng = np.random.default_rng(12)
    cell = _random_blocks(12)
    nz, ny, nx = cell.shape
    L = oracle_mod.Lattice(nx, ny, nz, 0.9, cell=cell)
    f = L.init(1.0, (0.01, 0.02, -0.01)) * (1 + 0.05 * rng.uniform(-1, 1, L.shape))
    g = L.step(f)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([x, y, z]).reshape(3, -1)
    syms = cube_symmetries()
    for i in rng.choice(len(syms), 6, replace=False):
        R = syms[i]
        nd = np.abs(R) @ np.array([nx, ny, nz])
        p2 = R @ pos
        for a in range(3):
            if (R[a] < 0).any():
                p2[a] += nd[a] - 1
        perm = population_perm(R)

        def tr(h):
            out = np.empty((19, nd[2], nd[1], nd[0]))
            for k in range(19):
                out[perm[k], p2[2], p2[1], p2[0]] = h[k].reshape(-1)
            return out

        c2 = np.empty((nd[2], nd[1], nd[0]), np.uint8)
        c2[p2[2], p2[1], p2[0]] = cell.reshape(-1)
        L2 = oracle_mod.Lattice(int(nd[0]), int(nd[1]), int(nd[2]), 0.9, cell=c2)
        a_ = L2.step(tr(f))
        b_ = tr(g)
        live = c2 != 2
        np.testing.assert_allclose(a_[:, live], b_[:, live], rtol=0, atol=1e-15)
