"""Helpers for tests: the 48 symmetries of the cube acting on the D3Q19
lattice, built from the paper's printed matrix M (eq_deffs).

A symmetry R (a signed 3x3 permutation matrix) maps every lattice vector c_i
to another one, R c_i = c_{p(i)}; a population array f transforms as
g[p(i)] = f[i], a velocity as R v, and a face with inward normal n goes to the
face with inward normal R n.  Test support only: no arithmetic of the method.
"""
import itertools
import os

import numpy as np

_M = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "d3q19_matrix_M.txt"), comments="#")
C = _M.T.astype(int)  # (19, 3)
NORMALS = np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])


def cube_symmetries():
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=int)
            for a in range(3):
                R[a, perm[a]] = signs[a]
            out.append(R)
    return out


def population_perm(R):
    """p with R c_i = c_{p[i]}."""
    p = np.empty(19, dtype=int)
    for i, ci in enumerate(C):
        rc = R @ ci
        p[i] = int(np.flatnonzero((C == rc).all(axis=1))[0])
    return p


def face_of_normal(n):
    return int(np.flatnonzero((NORMALS == np.asarray(n)).all(axis=1))[0])


def apply_to_pops(R, f):
    p = population_perm(R)
    g = np.empty_like(f)
    g[p] = f
    return g
