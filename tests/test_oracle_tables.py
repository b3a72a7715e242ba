"""Pins of the oracle's lattice tables and equilibrium against what the paper
prints (eq_deffs, eq_weights) and what the mathematics fixes (moments of
eq_feq)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def paper_c():
    """Lattice vectors from the printed matrix M (eq_deffs), shape (19, 3)."""
    return _golden("d3q19_matrix_M.txt").T.astype(int)


def paper_w():
    return _golden("d3q19_weights.txt") / 36.0


def test_velocity_table_matches_paper_matrix(oracle_mod):
    c, _ = oracle_mod.tables()
    np.testing.assert_array_equal(c, paper_c())


def test_weights_match_paper(oracle_mod):
    _, w = oracle_mod.tables()
    np.testing.assert_allclose(w, paper_w(), rtol=0, atol=1e-17)


def test_lattice_isotropy():
    # Closed forms every D3Q19 weight set must satisfy (c_s^2 = 1/3, Sec. II).
    c, w = paper_c(), paper_w()
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(w @ c, 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3.0, atol=1e-16)
    # Every vector has its opposite in the set.
    for ci in c:
        assert any((cj == -ci).all() for cj in c)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(oracle_mod, seed):
    # Moments of the second-order equilibrium (eq_feq): rho, rho u and
    # rho/3 I + rho u u, exactly (up to rounding).
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0)
    u = rng.uniform(-0.1, 0.1, 3)
    c = paper_c()
    feq = oracle_mod.feq(rho, u)
    assert abs(feq.sum() - rho) < 1e-14
    np.testing.assert_allclose(feq @ c, rho * u, atol=1e-15)
    pi = np.einsum("i,ia,ib->ab", feq, c, c)
    np.testing.assert_allclose(pi, rho / 3.0 * np.eye(3) + rho * np.outer(u, u), atol=1e-15)


def test_equilibrium_at_rest_is_weights(oracle_mod):
    np.testing.assert_allclose(oracle_mod.feq(1.7, (0, 0, 0)), 1.7 * paper_w(), rtol=1e-15)
