"""Host-only cross-check (no GPU) of the library's complex-geometry
classification (lbm_classify_geometry) against the oracle's; the two are
written independently.  Each wall node must get the same unknown set and the
same rule kind: plane, concave edge or corner (with the wall planes as a face
mask), convex edge, or the general rule."""
import numpy as np
import pytest

from paper_0811_4593_amd import workloads
from test_oracle_complex_geometry import _box_geometry, _random_blocks


def _oracle_codes(oracle_mod, L, cell):
    kinds = np.full(cell.shape, -1)
    unk = np.zeros(cell.shape, np.int64)
    for z, y, x in zip(*np.nonzero(cell == 1)):
        kinds[z, y, x], unk[z, y, x] = L.classify(x, y, z)
    return kinds, unk


@pytest.mark.parametrize("case", ["box", "rib", "blocks", "noise"])
def test_library_classification_matches_oracle(oracle_mod, case):
    from paper_0811_4593_amd import lbm
    if case == "box":
        cell = _box_geometry(6, 5, 4)
    elif case == "rib":
        cell = workloads.rib_channel()[1]
    elif case == "blocks":
        cell = _random_blocks(12)
    else:
        rng = np.random.default_rng(3)
        cell = workloads.cells_from_solid(rng.uniform(size=(9, 8, 11)) < 0.35)
    nz, ny, nx = cell.shape
    L = oracle_mod.Lattice(nx, ny, nz, 0.8, cell=cell)
    kinds, unk = _oracle_codes(oracle_mod, L, cell)
    code, counts = lbm.lbm_classify_geometry(cell)
    lib_kind = code >> 24
    lib_m = (code >> 18) & 63
    lib_u = code & 0x3FFFF
    wall = cell == 1
    np.testing.assert_array_equal(lib_u[wall], unk[wall])
    expect = np.select([kinds == oracle_mod.NODE_FLUID, kinds == oracle_mod.NODE_FACE, kinds == oracle_mod.NODE_EDGE,
                        kinds == oracle_mod.NODE_CORNER, kinds == oracle_mod.NODE_CONVEX_EDGE,
                        kinds == oracle_mod.NODE_GENERAL], [lbm.GEO_FLUID, lbm.GEO_PLANE_EDGE_CORNER,
                                                             lbm.GEO_PLANE_EDGE_CORNER, lbm.GEO_PLANE_EDGE_CORNER,
                                                             lbm.GEO_CONVEX_EDGE, lbm.GEO_GENERAL], -1)
    np.testing.assert_array_equal(lib_kind[wall], expect[wall])
    walls_count = np.array([bin(int(m)).count("1") for m in lib_m[wall]])
    for k, nw in ((oracle_mod.NODE_FACE, 1), (oracle_mod.NODE_EDGE, 2), (oracle_mod.NODE_CORNER, 3)):
        assert (walls_count[kinds[wall] == k] == nw).all()
    assert (lib_kind[cell == 2] == lbm.GEO_SOLID).all() and (lib_kind[cell == 0] == lbm.GEO_FLUID).all()
    assert sum(counts) == cell.size
    if case == "blocks":
        assert counts[lbm.GEO_GENERAL] > 0 and counts[lbm.GEO_CONVEX_EDGE] > 0
