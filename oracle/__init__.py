"""Plain FP64 CPU oracle for the D3Q19 on-site Zou-He step (Hecht & Harting,
arXiv:0811.4593).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s ``cpu_baseline`` leg may import this package.  It wraps the C
code in ``d3q19_oracle.c`` (compiled by ``oracle.build``) with ctypes and numpy
and shares nothing with the HIP library in ``paper_0811_4593_amd``.

Conventions: node index n = x + nx*(y + ny*z); population k = i - 1 in the
paper's numbering (Sec. II, eq_deffs); state arrays are float64 of shape
(19, nz, ny, nx); faces 0..5 are x=0, x=nx-1, y=0, y=ny-1, z=0, z=nz-1.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)


class _OracleLattice(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("bc_set", ctypes.c_int * 6),
        ("v", (ctypes.c_double * 3) * 6),
        ("force", ctypes.c_double * 3),
        ("bc_pressure", ctypes.c_int * 6),
        ("rho_bc", ctypes.c_double * 6),
        ("solid", ctypes.POINTER(ctypes.c_ubyte)),
        ("face_v", _dp * 6),
        ("no_transverse", ctypes.c_int),
        ("cell", ctypes.POINTER(ctypes.c_ubyte)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.oracle_tables.argtypes = [ctypes.POINTER(ctypes.c_int), _dp]
        lib.oracle_feq.argtypes = [ctypes.c_double, _dp, _dp]
        lib.oracle_face_rule.argtypes = [ctypes.c_int, _dp, _dp]
        lib.oracle_edge_rule.argtypes = [ctypes.c_int, ctypes.c_int, _dp]
        lib.oracle_corner_rule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        lib.oracle_face_rule_no_transverse.argtypes = [ctypes.c_int, _dp, _dp]
        lib.oracle_convex_edge_rule.argtypes = [ctypes.c_int, ctypes.c_int, _dp]
        lib.oracle_general_rule.argtypes = [ctypes.c_uint, _dp]
        lib.oracle_classify.argtypes = [ctypes.POINTER(_OracleLattice), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_uint)]
        lib.oracle_classify.restype = ctypes.c_int
        lib.oracle_face_rule_pressure.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        lib.oracle_edge_rule_pressure.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
        lib.oracle_corner_rule_pressure.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                    _dp]
        lib.oracle_update_node.argtypes = [ctypes.POINTER(_OracleLattice), ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, _dp, _dp, _dp]
        lib.oracle_update_node.restype = ctypes.c_int
        lib.oracle_init.argtypes = [ctypes.POINTER(_OracleLattice), ctypes.c_double, _dp, _dp]
        lib.oracle_step.argtypes = [ctypes.POINTER(_OracleLattice), _dp, _dp, _dp, ctypes.c_int]
        lib.oracle_step.restype = ctypes.c_int
        lib.oracle_moments.argtypes = [ctypes.POINTER(_OracleLattice), _dp, _dp, _dp]
        lib.oracle_totals.argtypes = [ctypes.POINTER(_OracleLattice), _dp, _dp, _dp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _vec(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))


# Face numbering and inward normals (same order as the oracle's C code).
FACES = ("x0", "x1", "y0", "y1", "z0", "z1")
NORMALS = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def tables():
    """Return (c[19,3] int, w[19] float64) as the oracle holds them."""
    lib = _load()
    c = (ctypes.c_int * 57)()
    w = np.zeros(19)
    lib.oracle_tables(c, _ptr(w))
    return np.array(list(c), dtype=np.int64).reshape(19, 3), w


def feq(rho: float, u) -> np.ndarray:
    lib = _load()
    out = np.zeros(19)
    lib.oracle_feq(float(rho), _ptr(_vec(u)), _ptr(out))
    return out


def face_rule(face: int, v, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_face_rule(int(face), _ptr(_vec(v)), _ptr(g))
    return g


def edge_rule(face_a: int, face_b: int, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_edge_rule(int(face_a), int(face_b), _ptr(g))
    return g


def corner_rule(face_a: int, face_b: int, face_c: int, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_corner_rule(int(face_a), int(face_b), int(face_c), _ptr(g))
    return g


def face_rule_no_transverse(face: int, v, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_face_rule_no_transverse(int(face), _ptr(_vec(v)), _ptr(g))
    return g


def convex_edge_rule(face_a: int, face_b: int, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_convex_edge_rule(int(face_a), int(face_b), _ptr(g))
    return g


def general_rule(unknown: int, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_general_rule(int(unknown), _ptr(g))
    return g


# Rule kinds of wall nodes (oracle_classify).
NODE_FLUID, NODE_FACE, NODE_EDGE, NODE_CORNER, NODE_CONVEX_EDGE, NODE_GENERAL = range(6)


def face_rule_pressure(face: int, rho0: float, v, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_face_rule_pressure(int(face), float(rho0), _ptr(_vec(v)), _ptr(g))
    return g


def edge_rule_pressure(face_a: int, face_b: int, rho0: float, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_edge_rule_pressure(int(face_a), int(face_b), float(rho0), _ptr(g))
    return g


def corner_rule_pressure(face_a: int, face_b: int, face_c: int, rho0: float, f) -> np.ndarray:
    lib = _load()
    g = _vec(f).copy()
    lib.oracle_corner_rule_pressure(int(face_a), int(face_b), int(face_c), float(rho0), _ptr(g))
    return g


@dataclass
class Lattice:
    """A lattice description for the oracle: size, tau, face BCs, body force.

    bc: face -> prescribed velocity (velocity faces), or the tangential
    velocity of a pressure face; pressure: face -> prescribed density (the
    face becomes a pressure face; its tangential velocity is bc.get(face, 0)).
    solid: optional (nz, ny, nx) bool/uint8 array of solid nodes (mid-grid
    bounce-back); face_v: face -> per-node velocities of a velocity face,
    shape (n2, n1, 3) over the face's two other axes (z faces: (ny, nx, 3),
    y faces: (nz, nx, 3), x faces: (nz, ny, 3)); no_transverse: the face rule
    without the transverse corrections (comparison variant).  cell: optional
    (nz, ny, nx) node types for complex geometry: 0 fluid, 1 wall node
    (on-site no-slip), 2 solid interior; every axis periodic then."""

    nx: int
    ny: int
    nz: int
    tau: float
    bc: dict = field(default_factory=dict)  # face index -> velocity (3,)
    force: tuple = (0.0, 0.0, 0.0)
    pressure: dict = field(default_factory=dict)  # face index -> rho0
    solid: np.ndarray | None = None
    face_v: dict = field(default_factory=dict)  # face index -> per-node velocities
    no_transverse: bool = False
    cell: np.ndarray | None = None

    @property
    def shape(self):
        return (19, self.nz, self.ny, self.nx)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def _c(self) -> _OracleLattice:
        s = _OracleLattice()
        s.nx, s.ny, s.nz, s.tau = self.nx, self.ny, self.nz, float(self.tau)
        for face, v in self.bc.items():
            s.bc_set[face] = 1
            for a in range(3):
                s.v[face][a] = float(v[a])
        for face, rho0 in self.pressure.items():
            s.bc_set[face] = 1
            s.bc_pressure[face] = 1
            s.rho_bc[face] = float(rho0)
        for a in range(3):
            s.force[a] = float(self.force[a])
        keep = []
        if self.solid is not None:
            sol = np.ascontiguousarray(np.asarray(self.solid).astype(np.uint8).reshape(self.nz, self.ny, self.nx))
            keep.append(sol)
            s.solid = sol.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
        for face, fv in self.face_v.items():
            a = np.ascontiguousarray(np.asarray(fv, dtype=np.float64))
            n_face = {0: self.ny * self.nz, 1: self.nx * self.nz, 2: self.nx * self.ny}[face // 2]
            assert a.size == 3 * n_face, "face velocity field has the wrong size"
            keep.append(a)
            s.bc_set[face] = 1
            s.face_v[face] = a.ctypes.data_as(_dp)
        s.no_transverse = int(bool(self.no_transverse))
        if self.cell is not None:
            cel = np.ascontiguousarray(np.asarray(self.cell).astype(np.uint8).reshape(self.nz, self.ny, self.nx))
            keep.append(cel)
            s.cell = cel.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
        self._keep = keep  # the C struct points into these arrays
        return s

    def init(self, rho0: float = 1.0, u0=(0.0, 0.0, 0.0)) -> np.ndarray:
        f = np.empty(self.shape)
        _load().oracle_init(ctypes.byref(self._c()), float(rho0), _ptr(_vec(u0)), _ptr(f))
        return f

    def step(self, f: np.ndarray, nthreads: int = 0, want_u_pre: bool = False):
        """One step: pull streaming, boundary rules, BGK.  Returns the new
        state, or (state, u_pre[3,nz,ny,nx]) if want_u_pre."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == self.shape
        out = np.empty_like(f)
        up = np.empty((3, self.nz, self.ny, self.nx)) if want_u_pre else None
        rc = _load().oracle_step(ctypes.byref(self._c()), _ptr(f), _ptr(out), _ptr(up), int(nthreads))
        if rc != 0:
            raise ValueError("invalid lattice description for the oracle")
        return (out, up) if want_u_pre else out

    def run(self, f: np.ndarray, steps: int, nthreads: int = 0) -> np.ndarray:
        for _ in range(steps):
            f = self.step(f, nthreads)
        return f

    def update_node(self, x: int, y: int, z: int, pulled) -> np.ndarray:
        out = np.zeros(19)
        rc = _load().oracle_update_node(ctypes.byref(self._c()), int(x), int(y), int(z),
                                        _ptr(_vec(pulled)), _ptr(out), None)
        if rc != 0:
            raise ValueError("invalid lattice description for the oracle")
        return out

    def classify(self, x: int, y: int, z: int):
        """(rule kind, unknown bit set) of a wall node, or (-1, 0)."""
        u = ctypes.c_uint(0)
        k = _load().oracle_classify(ctypes.byref(self._c()), int(x), int(y), int(z), ctypes.byref(u))
        return k, u.value

    def moments(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        rho = np.empty((self.nz, self.ny, self.nx))
        u = np.empty((3, self.nz, self.ny, self.nx))
        _load().oracle_moments(ctypes.byref(self._c()), _ptr(f), _ptr(rho), _ptr(u))
        return rho, u

    def totals(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        m = ctypes.c_double()
        j = np.zeros(3)
        _load().oracle_totals(ctypes.byref(self._c()), _ptr(f), ctypes.byref(m), _ptr(j))
        return m.value, j
