"""Pins of the oracle's face rule (Sec. IV and Appendix) on random populations.

The oracle types the six faces' explicit formulas.  These tests check them
against things the paper fixes in other ways:
  * the prescribed velocity is met exactly and the density obeys the mass
    balance of eq_uin (Sec. IV: the velocity the rule yields is the imposed one);
  * the solution of the paper's Ansatz -- non-equilibrium bounce-back on every
    unknown plus two unknown transverse corrections N (eq_f5, eq_f9-eq_f17),
    closed by the moment equations (eq_rho, eq_vx-eq_vz) -- solved here as a
    linear system, not from the closed forms;
  * equilibrium in gives equilibrium out (the N vanish at equilibrium);
  * the six faces are images of each other under the cube's symmetries.
"""
import numpy as np
import pytest

from lattice_symmetry import C, NORMALS, apply_to_pops, cube_symmetries, face_of_normal


def _random_case(rng):
    f = rng.uniform(0.02, 0.12, 19)
    v = rng.uniform(-0.08, 0.08, 3)
    return f, v


def _unknown(face):
    return C @ NORMALS[face] > 0


@pytest.mark.parametrize("face", range(6))
@pytest.mark.parametrize("seed", range(4))
def test_prescribed_velocity_is_exact(oracle_mod, face, seed):
    f, v = _random_case(np.random.default_rng(100 * face + seed))
    g = oracle_mod.face_rule(face, v, f)
    rho = g.sum()
    np.testing.assert_allclose(g @ C / rho, v, rtol=0, atol=2e-16)
    # Known populations are left alone.
    known = ~_unknown(face)
    np.testing.assert_array_equal(g[known], f[known])
    # Mass balance (eq_uin): rho (1 - v.n) = sum of in-plane + 2 * outgoing.
    cn = C @ NORMALS[face]
    rhs = f[cn == 0].sum() + 2.0 * f[cn < 0].sum()
    assert abs(rho * (1.0 - v @ NORMALS[face]) - rhs) < 1e-15


@pytest.mark.parametrize("face", range(6))
def test_unknowns_are_never_read(oracle_mod, face):
    f, v = _random_case(np.random.default_rng(7 + face))
    f[_unknown(face)] = np.nan
    g = oracle_mod.face_rule(face, v, f)
    assert np.isfinite(g).all()


def _solve_ansatz(face, f, v):
    """Solve the paper's Ansatz for the five unknowns of a face.

    Unknowns: the five f_j with c_j.n > 0, the two transverse corrections N_a
    (one per tangential axis a) and rho.  Equations:
      normal link    f_j = f_{-j} + (2 w_j / c_s^2) rho c_j.v   (eq_f5)
      diagonals      f_j = f_{-j} + (rho/6) c_j.v - sgn(c_j[a]) N_a   (eq_f9-eq_f17)
      moments        sum f = rho, sum f c = rho v   (eq_rho, eq_vx-eq_vz)
    """
    n = NORMALS[face]
    unk = np.flatnonzero(C @ n > 0)
    tang = [a for a in range(3) if n[a] == 0]
    opp = [int(np.flatnonzero((C == -C[j]).all(axis=1))[0]) for j in range(19)]
    nu = len(unk)
    ncol = nu + 2 + 1  # f_unknown, N_a, N_b, rho
    A, b = [], []
    for r, j in enumerate(unk):
        row = np.zeros(ncol)
        row[r] = 1.0
        rhs = f[opp[j]]
        cv = C[j] @ v
        if (C[j] == n).all():
            row[-1] = -(2.0 * (2.0 / 36.0) * 3.0) * cv
        else:
            row[-1] = -cv / 6.0
            a = [t for t in tang if C[j][t] != 0][0]
            row[nu + tang.index(a)] = np.sign(C[j][a])
        A.append(row)
        b.append(rhs)
    known = np.ones(19, bool)
    known[unk] = False
    # mass
    row = np.zeros(ncol)
    row[:nu] = 1.0
    row[-1] = -1.0
    A.append(row)
    b.append(-f[known].sum())
    # momentum
    for al in range(3):
        row = np.zeros(ncol)
        row[:nu] = C[unk, al]
        row[-1] = -v[al]
        A.append(row)
        b.append(-(f[known] @ C[known, al]))
    A, b = np.array(A), np.array(b)
    assert np.linalg.matrix_rank(A) == ncol
    x, *_ = np.linalg.lstsq(A, b, rcond=None)
    assert np.abs(A @ x - b).max() < 1e-14  # the Ansatz system is consistent
    return unk, x[:nu], x[nu:nu + 2], x[-1]


@pytest.mark.parametrize("face", range(6))
@pytest.mark.parametrize("seed", range(4))
def test_matches_solution_of_paper_ansatz(oracle_mod, face, seed):
    f, v = _random_case(np.random.default_rng(1000 + 10 * face + seed))
    g = oracle_mod.face_rule(face, v, f)
    unk, fu, _, rho = _solve_ansatz(face, f, v)
    np.testing.assert_allclose(g[unk], fu, rtol=0, atol=1e-14)
    assert abs(g.sum() - rho) < 1e-14


@pytest.mark.parametrize("face", range(6))
def test_equilibrium_is_a_fixed_point(oracle_mod, face):
    rng = np.random.default_rng(50 + face)
    rho = rng.uniform(0.8, 1.3)
    v = rng.uniform(-0.08, 0.08, 3)
    feq = oracle_mod.feq(rho, v)
    f = feq.copy()
    f[_unknown(face)] = rng.uniform(0, 1, _unknown(face).sum())
    g = oracle_mod.face_rule(face, v, f)
    np.testing.assert_allclose(g, feq, rtol=0, atol=1e-15)
    # With the corrections N forced to zero the result would differ from f^eq
    # only through N, so the fixed point also shows N = 0 at equilibrium.


@pytest.mark.parametrize("face", range(6))
def test_faces_are_symmetric_images(oracle_mod, face):
    rng = np.random.default_rng(77 + face)
    for R in cube_symmetries():
        f, v = _random_case(rng)
        g = oracle_mod.face_rule(face, v, f)
        face2 = face_of_normal(R @ NORMALS[face])
        g2 = oracle_mod.face_rule(face2, R @ v, apply_to_pops(R, f))
        np.testing.assert_allclose(g2, apply_to_pops(R, g), rtol=0, atol=1e-15)


def test_no_slip_face_is_node_bounce_back_plus_correction(oracle_mod):
    # v = 0 on the bottom plane: f5 = f6 exactly (eq_f5 with v_z = 0) and the
    # diagonals differ from plain bounce-back only by the corrections N.
    rng = np.random.default_rng(5)
    f = rng.uniform(0.02, 0.12, 19)
    g = oracle_mod.face_rule(4, (0, 0, 0), f)
    # paper indices 5 <- 6, 9 <- 14, 13 <- 10, 15 <- 18, 17 <- 16  (k = i - 1)
    assert g[4] == f[5]
    nzx = g[8] - f[13]
    nzy = g[14] - f[17]
    assert abs((g[12] - f[9]) + nzx) < 1e-16
    assert abs((g[16] - f[15]) + nzy) < 1e-16
