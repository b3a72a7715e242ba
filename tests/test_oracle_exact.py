"""Exact rational brute force of whole steps on a tiny lattice (no GPU).

A 4 x 4 x 4 lattice bounded on all six faces (moving walls with rational
velocities) holds every node class: 24 face nodes, 24 edge nodes, 8 corners
and 8 bulk nodes.  Two steps are computed in exact arithmetic (Python
fractions) from the definitions, structured differently from the oracle:

  * streaming pulls f_i(x - c_i); a source outside the lattice is unknown;
  * a face node's five unknowns, the two transverse corrections and the
    density are the exact solution of the paper's Ansatz as a linear system
    (non-equilibrium bounce-back with corrections N, eq_f5, eq_f9-eq_f17,
    plus mass and momentum, eq_rho, eq_vx-eq_vz), solved by Gaussian
    elimination over the rationals;
  * an edge node bounces back its unknowns but the buried pair, then the four
    bounced populations along the edge take equal shares of the edge momentum
    with the sign that cancels it, and the buried pair and the rest
    population are fixed by reproducing the rest state's weights (Sec. V);
    a corner node likewise, without the correction;
  * BGK with the second-order equilibrium, tau = 4/5.

The oracle (FP64) must agree to rounding: 1e-14 relative after each step.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from lattice_symmetry import C, NORMALS

W = [Fr(2, 36)] * 6 + [Fr(1, 36)] * 12 + [Fr(12, 36)]
OPP = [int(np.flatnonzero((C == -c).all(axis=1))[0]) for c in C]
CL = [tuple(int(a) for a in c) for c in C]
NL = [tuple(int(a) for a in n) for n in NORMALS]
SIZE = 4
TAU = Fr(4, 5)
V = {0: (Fr(1, 50), Fr(1, 100), Fr(-1, 100)), 1: (Fr(-1, 100), Fr(1, 50), Fr(1, 100)),
     2: (Fr(1, 100), Fr(1, 40), Fr(-1, 50)), 3: (Fr(1, 50), Fr(-1, 100), Fr(1, 100)),
     4: (Fr(-1, 50), Fr(1, 100), Fr(3, 100)), 5: (Fr(1, 100), Fr(-1, 50), Fr(-1, 100))}


def dot(a, b):
    return sum(x * y for x, y in zip(a, b))


def feq(rho, u):
    uu = dot(u, u)
    return [W[i] * rho * (1 + 3 * dot(CL[i], u) + Fr(9, 2) * dot(CL[i], u) ** 2 - Fr(3, 2) * uu) for i in range(19)]


def solve_exact(A, b):
    """Least-squares-free exact solve of a consistent over-determined system:
    Gaussian elimination with row swaps on [A | b]; checks consistency."""
    m, n = len(A), len(A[0])
    M = [row[:] + [bb] for row, bb in zip(A, b)]
    r = 0
    piv = []
    for c in range(n):
        p = next((i for i in range(r, m) if M[i][c] != 0), None)
        assert p is not None, "singular"
        M[r], M[p] = M[p], M[r]
        inv = 1 / M[r][c]
        M[r] = [x * inv for x in M[r]]
        for i in range(m):
            if i != r and M[i][c] != 0:
                fac = M[i][c]
                M[i] = [x - fac * y for x, y in zip(M[i], M[r])]
        piv.append(c)
        r += 1
    for i in range(r, m):
        assert M[i][n] == 0, "inconsistent Ansatz system"
    return [M[i][n] for i in range(n)]


def face_rule(f, face, v=None):
    n = NL[face]
    v = V[face] if v is None else v
    unk = [j for j in range(19) if dot(CL[j], n) > 0]
    tang = [a for a in range(3) if n[a] == 0]
    nu = len(unk)
    ncol = nu + 3  # unknown f, N_a, N_b, rho
    A, b = [], []
    for r, j in enumerate(unk):
        row = [Fr(0)] * ncol
        row[r] = Fr(1)
        cv = dot(CL[j], v)
        if CL[j] == n:
            row[-1] = -2 * W[j] * 3 * cv               # f_j = f_-j + (2 w / c_s^2) rho c_j.v
        else:
            row[-1] = -cv / 6
            a = next(t for t in tang if CL[j][t] != 0)
            row[nu + tang.index(a)] = Fr(CL[j][a])   # ... - sgn(c_j[a]) N_a
        A.append(row)
        b.append(f[OPP[j]])
    known = [i for i in range(19) if i not in unk]
    row = [Fr(1)] * nu + [Fr(0), Fr(0), Fr(-1)]
    A.append(row)
    b.append(-sum(f[i] for i in known))
    for al in range(3):
        row = [Fr(CL[j][al]) for j in unk] + [Fr(0), Fr(0), -v[al]]
        A.append(row)
        b.append(-sum(f[i] * CL[i][al] for i in known))
    x = solve_exact(A, b)
    g = f[:]
    for r, j in enumerate(unk):
        g[j] = x[r]
    return g


def face_rule_pressure(f, face, rho0):
    """Pressure face (eq_rhoin, Appendix): the density rho0 and the tangential
    velocity V[face] minus its normal part are given; the unknowns are the
    five populations, N_a, N_b and the normal velocity v_n, from the same
    bounce-back Ansatz plus mass and momentum."""
    n = NL[face]
    vt = tuple(V[face][a] - dot(V[face], n) * n[a] for a in range(3))
    unk = [j for j in range(19) if dot(CL[j], n) > 0]
    tang = [a for a in range(3) if n[a] == 0]
    nu = len(unk)
    ncol = nu + 3  # unknown f, N_a, N_b, v_n
    A, b = [], []
    for r, j in enumerate(unk):
        row = [Fr(0)] * ncol
        row[r] = Fr(1)
        # f_j - 6 w_j rho0 (c_j.n) v_n [+ sgn N] = f_-j + 6 w_j rho0 c_j.v_t
        row[-1] = -6 * W[j] * rho0 * dot(CL[j], n)
        if CL[j] != n:
            a = next(t for t in tang if CL[j][t] != 0)
            row[nu + tang.index(a)] = Fr(CL[j][a])
        A.append(row)
        b.append(f[OPP[j]] + 6 * W[j] * rho0 * dot(CL[j], vt))
    known = [i for i in range(19) if i not in unk]
    A.append([Fr(1)] * nu + [Fr(0)] * 3)
    b.append(rho0 - sum(f[i] for i in known))
    for al in range(3):
        A.append([Fr(CL[j][al]) for j in unk] + [Fr(0), Fr(0), -rho0 * n[al]])
        b.append(rho0 * vt[al] - sum(f[i] * CL[i][al] for i in known))
    x = solve_exact(A, b)
    g = f[:]
    for r, j in enumerate(unk):
        g[j] = x[r]
    return g


def wall_rule(f, faces, rho0=None):
    """Edge (two faces) or corner (three), walls at rest; next to a pressure
    plane (rho0 given) the buried links and the rest population share what
    the prescribed density leaves, in the ratio of their weights."""
    ns = [NL[fc] for fc in faces]
    unknown = [any(dot(CL[i], n) > 0 for n in ns) for i in range(18)]
    buried = [unknown[i] and unknown[OPP[i]] for i in range(18)]
    g = f[:]
    for i in range(18):
        if unknown[i] and not buried[i]:
            g[i] = f[OPP[i]]
    if len(faces) == 2:
        e = tuple(int(a) for a in np.cross(ns[0], ns[1]))
        P = sum(g[i] * dot(CL[i], e) for i in range(18) if not buried[i])
        along = [i for i in range(18) if unknown[i] and not buried[i] and dot(CL[i], e) != 0]
        assert len(along) == 4
        for i in along:  # equal shares of the edge momentum, cancelling it
            g[i] -= Fr(dot(CL[i], e)) * P / 4
    # buried links and rest: the value that returns a fluid at rest unchanged,
    # w_b / (sum of the other moving weights) times their sum; or, next to a
    # pressure plane, the node's density made rho0
    s = sum(g[i] for i in range(18) if not buried[i])
    ws = sum(W[i] for i in range(18) if not buried[i])
    share = s / ws if rho0 is None else (rho0 - s) / (1 - ws)
    for i in range(18):
        if buried[i]:
            g[i] = W[i] * share
    g[18] = W[18] * share
    return g


def exact_step(F, pressure=None):
    """F[z][y][x] -> list of 19 Fractions (post-collision).  pressure: face ->
    prescribed density of the pressure faces."""
    pressure = pressure or {}
    out = [[[None] * SIZE for _ in range(SIZE)] for _ in range(SIZE)]
    for z in range(SIZE):
        for y in range(SIZE):
            for x in range(SIZE):
                f = [None] * 19
                for i in range(19):
                    sx, sy, sz = x - CL[i][0], y - CL[i][1], z - CL[i][2]
                    if 0 <= sx < SIZE and 0 <= sy < SIZE and 0 <= sz < SIZE:
                        f[i] = F[sz][sy][sx][i]
                faces = [fc for fc, (a, lo) in enumerate([(0, 1), (0, 0), (1, 1), (1, 0), (2, 1), (2, 0)])
                         if (x, y, z)[a] == (0 if lo else SIZE - 1)]
                rho0 = next((pressure[fc] for fc in faces if fc in pressure), None)
                if len(faces) == 1:
                    f = face_rule(f, faces[0]) if rho0 is None else face_rule_pressure(f, faces[0], rho0)
                elif len(faces) >= 2:
                    f = wall_rule(f, faces, rho0)
                assert all(v is not None for v in f)
                rho = sum(f)
                u = tuple(sum(f[i] * CL[i][a] for i in range(19)) / rho for a in range(3))
                fe = feq(rho, u)
                out[z][y][x] = [f[i] - (f[i] - fe[i]) / TAU for i in range(19)]
    return out


def test_two_steps_exact_against_oracle(oracle_mod):
    rng = np.random.default_rng(3)
    # a rational start state: equilibrium of a small flow plus rational noise
    base = feq(Fr(1), (Fr(1, 100), Fr(-1, 50), Fr(1, 40)))
    F = [[[[base[i] * (1 + Fr(int(rng.integers(-50, 51)), 1000)) for i in range(19)]
           for _ in range(SIZE)] for _ in range(SIZE)] for _ in range(SIZE)]
    L = oracle_mod.Lattice(SIZE, SIZE, SIZE, float(TAU), bc={fc: tuple(float(a) for a in V[fc]) for fc in range(6)})
    f_or = np.array([[[[float(F[z][y][x][i]) for x in range(SIZE)] for y in range(SIZE)] for z in range(SIZE)]
                     for i in range(19)])
    for _ in range(2):
        F = exact_step(F)
        f_or = L.step(f_or)
        exact = np.array([[[[float(F[z][y][x][i]) for x in range(SIZE)] for y in range(SIZE)] for z in range(SIZE)]
                          for i in range(19)])
        assert np.max(np.abs(f_or - exact) / np.abs(exact)) < 1e-14


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_two_steps_exact_with_pressure_faces_against_oracle(oracle_mod, axis):
    """The same lattice with the two faces of one axis as pressure faces
    (densities 51/50 and 49/50, tangential velocities from V): the pressure
    face rule of all six faces (the normal velocity solved for), pressure
    edges and corners."""
    rng = np.random.default_rng(4 + axis)
    pressure = {2 * axis: Fr(51, 50), 2 * axis + 1: Fr(49, 50)}
    base = feq(Fr(1), (Fr(1, 100), Fr(-1, 50), Fr(1, 40)))
    F = [[[[base[i] * (1 + Fr(int(rng.integers(-50, 51)), 1000)) for i in range(19)]
           for _ in range(SIZE)] for _ in range(SIZE)] for _ in range(SIZE)]
    L = oracle_mod.Lattice(SIZE, SIZE, SIZE, float(TAU), bc={fc: tuple(float(a) for a in V[fc]) for fc in range(6)},
                           pressure={fc: float(r) for fc, r in pressure.items()})
    f_or = np.array([[[[float(F[z][y][x][i]) for x in range(SIZE)] for y in range(SIZE)] for z in range(SIZE)]
                     for i in range(19)])
    for _ in range(2):
        F = exact_step(F, pressure)
        f_or = L.step(f_or)
        exact = np.array([[[[float(F[z][y][x][i]) for x in range(SIZE)] for y in range(SIZE)] for z in range(SIZE)]
                          for i in range(19)])
        assert np.max(np.abs(f_or - exact) / np.abs(exact)) < 1e-14
    # every node of a pressure plane (edges and corners included) carries
    # its density exactly: the stored post-collision state keeps its mass
    rho = np.moveaxis(exact.sum(axis=0), 2 - axis, 0)  # (plane axis, ...)
    assert np.allclose(rho[0], 51 / 50, rtol=0, atol=1e-15)
    assert np.allclose(rho[-1], 49 / 50, rtol=0, atol=1e-15)


def _rule_at_rest(f, faces):
    """Face rule (exact Ansatz solve) for a wall at rest, or the edge/corner
    rule, for the walls `faces` (inward normals NL)."""
    if len(faces) == 1:
        saved = V[faces[0]]
        V[faces[0]] = (Fr(0), Fr(0), Fr(0))
        try:
            return face_rule(f, faces[0])
        finally:
            V[faces[0]] = saved
    return wall_rule(f, faces)


def exact_step_cells(F, cell):
    """One step of a periodic box with a complex geometry (Sec. V): cell 0
    fluid, 1 wall node (on-site no-slip), 2 solid interior (kept as is).  At
    a wall node the unknown populations are those arriving from solid
    interior; the walls are the planes all of whose incoming populations are
    unknown; the rule follows from that set: one plane, two (concave edge)
    or three (corner) orthogonal planes covering exactly the unknowns take
    the box rules; a single unknown diagonal (convex edge) is bounced back
    and the momentum along the edge is removed in equal shares from the four
    populations with c.e != 0 that leave into the bulk; anything else is
    bounced back where the opposite is known, the rest sharing the mass of
    the others in the ratio of their weights."""
    nz, ny, nx = cell.shape
    out = [[[None] * nx for _ in range(ny)] for _ in range(nz)]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if cell[z, y, x] == 2:
                    out[z][y][x] = F[z][y][x][:]
                    continue
                f = [None] * 19
                unk = set()
                for i in range(19):
                    sx, sy, sz = (x - CL[i][0]) % nx, (y - CL[i][1]) % ny, (z - CL[i][2]) % nz
                    if cell[sz, sy, sx] == 2:
                        unk.add(i)
                    else:
                        f[i] = F[sz][sy][sx][i]
                if unk:
                    assert cell[z, y, x] == 1
                    walls = [fc for fc in range(6) if all(i in unk for i in range(18) if dot(CL[i], NL[fc]) > 0)]
                    covered = {i for i in range(18) for fc in walls if dot(CL[i], NL[fc]) > 0}
                    axes = {fc // 2 for fc in walls}
                    g = f[:]
                    if covered == unk and 1 <= len(walls) <= 3 and len(axes) == len(walls):
                        g = _rule_at_rest(f, walls)
                    elif not walls and len(unk) == 1 and sum(abs(a) for a in CL[next(iter(unk))]) == 2:
                        i0 = next(iter(unk))
                        g[i0] = f[OPP[i0]]
                        n1 = tuple(CL[i0][a] if a == min(a for a in range(3) if CL[i0][a]) else 0 for a in range(3))
                        n2 = tuple(CL[i0][a] - n1[a] for a in range(3))
                        e = tuple(int(v) for v in np.cross(n1, n2))
                        P = sum(g[j] * dot(CL[j], e) for j in range(18))
                        for i in range(18):
                            if dot(CL[i], e) != 0 and dot(CL[i], n1) + dot(CL[i], n2) == 1:
                                g[i] -= Fr(dot(CL[i], e)) * P / 4
                    else:
                        buried = {i for i in unk if OPP[i] in unk}
                        for i in unk - buried:
                            g[i] = f[OPP[i]]
                        s = sum(g[i] for i in range(18) if i not in buried)
                        ws = sum(W[i] for i in range(18) if i not in buried)
                        for i in buried:
                            g[i] = W[i] * s / ws
                        g[18] = W[18] * s / ws
                    f = g
                rho = sum(f)
                u = tuple(sum(f[i] * CL[i][a] for i in range(19)) / rho for a in range(3))
                fe = feq(rho, u)
                out[z][y][x] = [f[i] - (f[i] - fe[i]) / TAU for i in range(19)]
    return out


def test_one_step_exact_complex_geometry_against_oracle(oracle_mod):
    """A small ribbed channel (every kind of wall node: plane, concave edge,
    corner, convex edge, edge meeting a plane) in exact arithmetic against
    the oracle: one step from a perturbed flowing state, 1e-14."""
    from paper_0811_4593_amd import workloads
    spec, cell = workloads.rib_channel(nx=12, ny=8, nz=10, rib=(4, 7, 4), tau=float(TAU))
    L = oracle_mod.Lattice(spec.nx, spec.ny, spec.nz, float(TAU), cell=cell)
    kinds = {L.classify(x, y, z)[0] for z in range(spec.nz) for y in range(spec.ny) for x in range(spec.nx)
             if cell[z, y, x] == 1}
    assert {oracle_mod.NODE_FACE, oracle_mod.NODE_EDGE, oracle_mod.NODE_CORNER, oracle_mod.NODE_CONVEX_EDGE,
            oracle_mod.NODE_GENERAL} <= kinds
    rng = np.random.default_rng(5)
    base = feq(Fr(1), (Fr(1, 50), Fr(-1, 100), Fr(1, 100)))
    F = [[[[base[i] * (1 + Fr(int(rng.integers(-50, 51)), 1000)) for i in range(19)] for _ in range(spec.nx)]
          for _ in range(spec.ny)] for _ in range(spec.nz)]
    f_or = np.array([[[[float(F[z][y][x][i]) for x in range(spec.nx)] for y in range(spec.ny)] for z in range(spec.nz)]
                     for i in range(19)])
    F = exact_step_cells(F, cell)
    f_or = L.step(f_or)
    exact = np.array([[[[float(F[z][y][x][i]) for x in range(spec.nx)] for y in range(spec.ny)] for z in range(spec.nz)]
                      for i in range(19)])
    assert np.max(np.abs(f_or - exact) / np.abs(exact)) < 1e-14


def face_rule_no_n(f, face):
    """Face rule without the transverse corrections (eq_f9NoNs-eq_f17NoNs):
    the density from mass and normal momentum (eq_uin), then every unknown
    is its opposite plus 6 w rho c.v."""
    n = NL[face]
    v = V[face]
    rho = (sum(f[i] for i in range(19) if dot(CL[i], n) == 0)
           + 2 * sum(f[i] for i in range(19) if dot(CL[i], n) < 0)) / (1 - dot(v, n))
    g = f[:]
    for j in range(19):
        if dot(CL[j], n) > 0:
            g[j] = f[OPP[j]] + 6 * W[j] * rho * dot(CL[j], v)
    return g


def exact_step_options(F, periodic_x, solid, force, no_n):
    """Two-face-pair lattice (x periodic, y and z bounded), mid-grid
    bounce-back at solid nodes (a population from a solid node is the
    node's own opposite one of the previous step; solid nodes keep theirs,
    Sec. III), body force as the velocity shift tau F / rho in f^eq
    (eq_gravity), optionally the face rule without N."""
    out = [[[None] * SIZE for _ in range(SIZE)] for _ in range(SIZE)]
    bounded = [(1, 1), (1, 0), (2, 1), (2, 0)]  # (axis, low side) of faces 2..5
    for z in range(SIZE):
        for y in range(SIZE):
            for x in range(SIZE):
                if (x, y, z) in solid:
                    out[z][y][x] = F[z][y][x][:]
                    continue
                f = [None] * 19
                for i in range(19):
                    sx, sy, sz = (x - CL[i][0]) % SIZE, y - CL[i][1], z - CL[i][2]
                    if 0 <= sy < SIZE and 0 <= sz < SIZE:
                        f[i] = F[z][y][x][OPP[i]] if (sx, sy, sz) in solid else F[sz][sy][sx][i]
                faces = [2 + k for k, (a, lo) in enumerate(bounded) if (x, y, z)[a] == (0 if lo else SIZE - 1)]
                if len(faces) == 1:
                    f = face_rule_no_n(f, faces[0]) if no_n else face_rule(f, faces[0])
                elif len(faces) == 2:
                    f = wall_rule(f, faces)
                assert all(v is not None for v in f)
                rho = sum(f)
                u = tuple((sum(f[i] * CL[i][a] for i in range(19)) + TAU * force[a]) / rho for a in range(3))
                fe = feq(rho, u)
                out[z][y][x] = [f[i] - (f[i] - fe[i]) / TAU for i in range(19)]
    return out


@pytest.mark.parametrize("no_n", [False, True])
def test_two_steps_exact_with_force_solid_nodes_and_rule_variant(oracle_mod, no_n):
    rng = np.random.default_rng(6)
    solid = {(1, 1, 2), (2, 2, 1), (3, 1, 1)}
    force = (Fr(1, 1000), Fr(-1, 2000), Fr(1, 1500))
    base = feq(Fr(1), (Fr(1, 100), Fr(-1, 50), Fr(1, 40)))
    F = [[[[base[i] * (1 + Fr(int(rng.integers(-50, 51)), 1000)) for i in range(19)]
           for _ in range(SIZE)] for _ in range(SIZE)] for _ in range(SIZE)]
    mask = np.zeros((SIZE, SIZE, SIZE), np.uint8)
    for x, y, z in solid:
        mask[z, y, x] = 1
    L = oracle_mod.Lattice(SIZE, SIZE, SIZE, float(TAU), bc={fc: tuple(float(a) for a in V[fc]) for fc in range(2, 6)},
                           force=tuple(float(a) for a in force), solid=mask, no_transverse=no_n)
    f_or = np.array([[[[float(F[z][y][x][i]) for x in range(SIZE)] for y in range(SIZE)] for z in range(SIZE)]
                     for i in range(19)])
    for _ in range(2):
        F = exact_step_options(F, True, solid, force, no_n)
        f_or = L.step(f_or)
        exact = np.array([[[[float(F[z][y][x][i]) for x in range(SIZE)] for y in range(SIZE)] for z in range(SIZE)]
                          for i in range(19)])
        assert np.max(np.abs(f_or - exact) / np.abs(exact)) < 1e-14


def test_two_steps_exact_with_per_node_face_velocities(oracle_mod):
    """Velocity fields on the two x faces varying over y and z (face node
    order y + ny z, given to the oracle as (nz, ny, 3) arrays), uniform
    moving walls on y and z: the face rule takes each node's own velocity."""
    rng = np.random.default_rng(8)
    fields = {fc: [[tuple(Fr(int(rng.integers(-30, 31)), 1000) for _ in range(3)) for _ in range(SIZE)]
                   for _ in range(SIZE)] for fc in (0, 1)}  # [z][y] -> v
    base = feq(Fr(1), (Fr(1, 100), Fr(-1, 50), Fr(1, 40)))
    F = [[[[base[i] * (1 + Fr(int(rng.integers(-50, 51)), 1000)) for i in range(19)]
           for _ in range(SIZE)] for _ in range(SIZE)] for _ in range(SIZE)]
    face_v = {fc: np.array([[[float(a) for a in fields[fc][z][y]] for y in range(SIZE)] for z in range(SIZE)])
              for fc in (0, 1)}
    L = oracle_mod.Lattice(SIZE, SIZE, SIZE, float(TAU), bc={fc: tuple(float(a) for a in V[fc]) for fc in range(6)},
                           face_v=face_v)
    f_or = np.array([[[[float(F[z][y][x][i]) for x in range(SIZE)] for y in range(SIZE)] for z in range(SIZE)]
                     for i in range(19)])
    for _ in range(2):
        out = [[[None] * SIZE for _ in range(SIZE)] for _ in range(SIZE)]
        for z in range(SIZE):
            for y in range(SIZE):
                for x in range(SIZE):
                    f = [None] * 19
                    for i in range(19):
                        sx, sy, sz = x - CL[i][0], y - CL[i][1], z - CL[i][2]
                        if 0 <= sx < SIZE and 0 <= sy < SIZE and 0 <= sz < SIZE:
                            f[i] = F[sz][sy][sx][i]
                    faces = [fc for fc, (a, lo) in enumerate([(0, 1), (0, 0), (1, 1), (1, 0), (2, 1), (2, 0)])
                             if (x, y, z)[a] == (0 if lo else SIZE - 1)]
                    if len(faces) == 1:
                        v = fields[faces[0]][z][y] if faces[0] in fields else None
                        f = face_rule(f, faces[0], v)
                    elif len(faces) >= 2:
                        f = wall_rule(f, faces)
                    rho = sum(f)
                    u = tuple(sum(f[i] * CL[i][a] for i in range(19)) / rho for a in range(3))
                    fe = feq(rho, u)
                    out[z][y][x] = [f[i] - (f[i] - fe[i]) / TAU for i in range(19)]
        F = out
        f_or = L.step(f_or)
        exact = np.array([[[[float(F[z][y][x][i]) for x in range(SIZE)] for y in range(SIZE)] for z in range(SIZE)]
                          for i in range(19)])
        assert np.max(np.abs(f_or - exact) / np.abs(exact)) < 1e-14
