"""Pins of the oracle's no-slip edge and corner rules (Sec. V: eq_Nxzy,
eq_edge, eq_buried, eq_corner) on random populations.

What the paper fixes: the node velocity is zero after the rule (the purpose
of the rule is no-slip); the buried links take a common value chosen so that populations at
rest reproduce their lattice weights (the 22/36 and 18/36 counts); the rest
population is 12 times the buried value; for the edge the paper names the
corrected populations (7, 8, 15, 17 on the y-edge of the bottom and left
planes) and the correction's size (f3 - f4)/4; corners take no correction.
"""
import itertools

import numpy as np
import pytest

from lattice_symmetry import C, NORMALS, apply_to_pops, cube_symmetries, face_of_normal

EDGES = [(a, b) for a, b in itertools.combinations(range(6), 2) if a // 2 != b // 2]
CORNERS = [(a, b, c) for a in (0, 1) for b in (2, 3) for c in (4, 5)]
W = np.array([2] * 6 + [1] * 12 + [12]) / 36.0


def _known_mask(faces):
    m = np.ones(19, bool)
    for fc in faces:
        m &= C @ NORMALS[fc] <= 0
    m[18] = False  # the rest population is reassigned by the rule
    return m


def test_edge_and_corner_counts():
    assert len(EDGES) == 12 and len(CORNERS) == 8


@pytest.mark.parametrize("edge", EDGES)
def test_edge_velocity_is_zero(oracle_mod, edge):
    rng = np.random.default_rng(sum(edge))
    for _ in range(5):
        f = rng.uniform(0.02, 0.12, 19)
        g = oracle_mod.edge_rule(*edge, f)
        np.testing.assert_allclose(g @ C, 0.0, atol=1e-16)
        known = _known_mask(edge)
        np.testing.assert_array_equal(g[known], f[known])


@pytest.mark.parametrize("edge", EDGES)
def test_edge_unknowns_never_read(oracle_mod, edge):
    f = np.random.default_rng(3).uniform(0.02, 0.12, 19)
    unknown = ~_known_mask(edge)
    unknown[18] = False
    f[unknown] = np.nan
    assert np.isfinite(oracle_mod.edge_rule(*edge, f)).all()


@pytest.mark.parametrize("edge", EDGES)
def test_edge_rest_equilibrium_fixed_point(oracle_mod, edge):
    # Populations at rest, f = w rho: the rule must return them unchanged,
    # which fixes the divisor 22 and the factor 12 of eq_buried.
    rho = 1.37
    f = W * rho
    np.testing.assert_allclose(oracle_mod.edge_rule(*edge, f), f, rtol=1e-15)


@pytest.mark.parametrize("edge", EDGES)
def test_edge_buried_pair(oracle_mod, edge):
    a, b = edge
    n1, n2 = NORMALS[a], NORMALS[b]
    f = np.random.default_rng(11).uniform(0.02, 0.12, 19)
    g = oracle_mod.edge_rule(a, b, f)
    bur = [int(np.flatnonzero((C == s * (n1 - n2)).all(axis=1))[0]) for s in (1, -1)]
    assert g[bur[0]] == g[bur[1]]
    assert abs(g[18] - 12.0 * g[bur[0]]) < 1e-16
    # The buried value carries the 16 other moving populations' density at the
    # diagonal weight: 22 = 6*2 + 10*1 in units of 1/36.
    others = [k for k in range(18) if k not in bur]
    assert len(others) == 16
    assert abs(W[others].sum() - 22.0 / 36.0) < 1e-16
    assert abs(g[bur[0]] - g[others].sum() / 22.0) < 1e-16


def test_paper_edge_example(oracle_mod):
    # Edge of the bottom (z=0, face 4) and left (x=0, face 0) planes: the
    # y-axis.  After plain bounce-back the paper corrects exactly f7, f8, f15,
    # f17, each by (f3 - f4)/4 in magnitude.
    f = np.random.default_rng(21).uniform(0.02, 0.12, 19)
    g = oracle_mod.edge_rule(4, 0, f)
    opp = {i: int(np.flatnonzero((C == -C[i]).all(axis=1))[0]) for i in range(19)}
    plain = f.copy()
    for k in range(18):
        unknown = (C[k] @ NORMALS[4] > 0) or (C[k] @ NORMALS[0] > 0)
        buried = (C[k] == NORMALS[4] - NORMALS[0]).all() or (C[k] == NORMALS[0] - NORMALS[4]).all()
        if unknown and not buried:
            plain[k] = f[opp[k]]
    changed = [k + 1 for k in range(18) if abs(g[k] - plain[k]) > 1e-17 and not
               ((C[k] == NORMALS[4] - NORMALS[0]).all() or (C[k] == NORMALS[0] - NORMALS[4]).all())]
    assert changed == [7, 8, 15, 17]
    for i in changed:
        assert abs(abs(g[i - 1] - plain[i - 1]) - abs(f[2] - f[3]) / 4.0) < 1e-16


@pytest.mark.parametrize("corner", CORNERS)
def test_corner_velocity_zero_and_buried(oracle_mod, corner):
    s = NORMALS[list(corner)].sum(axis=0)
    buried = [k for k in range(18) if C[k] @ s == 0]
    assert len(buried) == 6
    rng = np.random.default_rng(sum(corner))
    for _ in range(5):
        f = rng.uniform(0.02, 0.12, 19)
        g = oracle_mod.corner_rule(*corner, f)
        np.testing.assert_allclose(g @ C, 0.0, atol=1e-16)
        known = _known_mask(corner)
        np.testing.assert_array_equal(g[known], f[known])
        assert np.ptp(g[buried]) == 0.0
        assert abs(g[18] - 12.0 * g[buried[0]]) < 1e-16
        others = [k for k in range(18) if k not in buried]
        assert abs(W[others].sum() - 18.0 / 36.0) < 1e-16
        assert abs(g[buried[0]] - g[others].sum() / 18.0) < 1e-16


@pytest.mark.parametrize("corner", CORNERS)
def test_corner_rest_equilibrium_fixed_point(oracle_mod, corner):
    f = W * 0.91
    np.testing.assert_allclose(oracle_mod.corner_rule(*corner, f), f, rtol=1e-15)


@pytest.mark.parametrize("corner", CORNERS)
def test_corner_unknowns_never_read(oracle_mod, corner):
    f = np.random.default_rng(4).uniform(0.02, 0.12, 19)
    unknown = ~_known_mask(corner)
    unknown[18] = False
    f[unknown] = np.nan
    assert np.isfinite(oracle_mod.corner_rule(*corner, f)).all()


def test_edges_and_corners_are_symmetric_images(oracle_mod):
    rng = np.random.default_rng(9)
    for R in cube_symmetries():
        for edge in EDGES:
            f = rng.uniform(0.02, 0.12, 19)
            g = oracle_mod.edge_rule(*edge, f)
            e2 = [face_of_normal(R @ NORMALS[fc]) for fc in edge]
            g2 = oracle_mod.edge_rule(*e2, apply_to_pops(R, f))
            np.testing.assert_allclose(g2, apply_to_pops(R, g), rtol=0, atol=1e-15)
        for corner in CORNERS:
            f = rng.uniform(0.02, 0.12, 19)
            g = oracle_mod.corner_rule(*corner, f)
            c2 = [face_of_normal(R @ NORMALS[fc]) for fc in corner]
            g2 = oracle_mod.corner_rule(*c2, apply_to_pops(R, f))
            np.testing.assert_allclose(g2, apply_to_pops(R, g), rtol=0, atol=1e-15)
