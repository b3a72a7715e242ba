"""Seeded synthetic workloads: lattice sizes, boundary velocities, relaxation
times and random perturbation fields.

This module holds no arithmetic of the method (no equilibria, no boundary
rules): it only describes inputs, so that the HIP path and the CPU oracle can
be driven with identical set-ups.  The paper uses no dataset; its workloads
are geometric set-ups (Sec. VI), reproduced here with their sizes and
velocity ranges.

Faces are numbered x0, x1, y0, y1, z0, z1 = 0..5.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class LatticeSpec:
    nx: int
    ny: int
    nz: int
    tau: float
    bc: dict = field(default_factory=dict)  # face -> (ux, uy, uz); pressure faces: tangential velocity
    rho0: float = 1.0
    name: str = ""
    pressure: dict = field(default_factory=dict)  # face -> prescribed density

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz


def couette(nx=16, ny=16, nz=32, u_top=0.05, tau=1.0) -> LatticeSpec:
    """Shear flow between on-site walls: x, y periodic, z0 at rest, z1 moving
    along x (the paper's shear test, Sec. VI)."""
    return LatticeSpec(nx, ny, nz, tau, {4: (0.0, 0.0, 0.0), 5: (u_top, 0.0, 0.0)},
                       name=f"couette_{nx}x{ny}x{nz}")


def duct(nx, ny, nz, u_in=(0.04, 0.01, 0.01), tau=0.8) -> LatticeSpec:
    """Duct: no-slip on-site walls on the y and z faces; the same oblique
    velocity prescribed on the inlet x0 and the outlet x1."""
    z = (0.0, 0.0, 0.0)
    u = tuple(float(a) for a in u_in)
    return LatticeSpec(nx, ny, nz, tau, {0: u, 1: u, 2: z, 3: z, 4: z, 5: z}, name=f"duct_{nx}x{ny}x{nz}")


def roofline_duct() -> LatticeSpec:
    """The 1024 x 512 x 512 duct, inlet/outlet (0.04, 0.01, 0.01), tau 0.8."""
    return duct(1024, 512, 512, (0.04, 0.01, 0.01), 0.8)


def precision_duct() -> LatticeSpec:
    """The same duct at 512 x 256 x 256 (storage-precision comparison)."""
    return duct(512, 256, 256, (0.04, 0.01, 0.01), 0.8)


def oblique_direction(rng: np.random.Generator):
    """Unit vector (1, a, b)/|(1, a, b)|, a, b ~ U[-0.5, 0.5] (inflow along +x)."""
    a, b = rng.uniform(-0.5, 0.5, 2)
    d = np.array([1.0, a, b])
    return d / np.linalg.norm(d)


def batch_ducts(count=64, seed=0):
    """Uneven ducts: Nx ~ U{32..256}, Ny, Nz ~ U{16..128}, |u| ~ U[0.01, 0.05]
    along an oblique direction, tau ~ U[0.6, 1.5]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nx = int(rng.integers(32, 257))
        ny = int(rng.integers(16, 129))
        nz = int(rng.integers(16, 129))
        speed = float(rng.uniform(0.01, 0.05))
        d = oblique_direction(rng)
        tau = float(rng.uniform(0.6, 1.5))
        s = duct(nx, ny, nz, tuple(speed * d), tau)
        s.name = f"batch{i}_{nx}x{ny}x{nz}"
        out.append(s)
    return out


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the trace
    spec: LatticeSpec
    storage: str    # "f32" or "f16sr"


def serving_trace(count=2000, rate=1.0, seed=1, n_min=16, n_max=256):
    """Poisson arrivals at `rate` per second of cubic ducts with N log-uniform
    in [n_min, n_max], |u| ~ U[0.01, 0.05] along an oblique direction,
    tau ~ U[0.6, 1.5], storage FP32 or FP16 with probability 1/2 each (the
    FP16 requests use stochastic rounding, the FP16 form that meets the 1e-3
    velocity bound at steady state)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        speed = float(rng.uniform(0.01, 0.05))
        d = oblique_direction(rng)
        tau = float(rng.uniform(0.6, 1.5))
        storage = "f16sr" if rng.uniform() < 0.5 else "f32"
        s = duct(n, n, n, tuple(speed * d), tau)
        s.name = f"req{i}_{n}^3"
        out.append(Request(i, t, s, storage))
    return out


def square_channel(n: int, tau: float = 1.0, drho: float = 1e-3) -> LatticeSpec:
    """Square channel n x n x (n + 1) (Sec. VI): no-slip walls on the x and y
    faces, pressure inlet z0 (density 1 + drho/2) and outlet z1 (1 - drho/2)."""
    w = (0.0, 0.0, 0.0)
    return LatticeSpec(n, n, n + 1, tau, {0: w, 1: w, 2: w, 3: w},
                       pressure={4: 1.0 + drho / 2, 5: 1.0 - drho / 2}, name=f"square_channel_{n}")


def pressure_classes_lattices():
    """Small lattices with pressure faces: every node class next to a pressure
    face, tangential velocities, a pressure inlet with a velocity outlet."""
    w = (0.0, 0.0, 0.0)
    return [
        LatticeSpec(7, 6, 8, 0.8, {0: w, 1: w, 2: w, 3: w}, pressure={4: 1.02, 5: 0.99}, name="pressure_duct_7x6x8"),
        LatticeSpec(9, 5, 6, 1.2, {0: (0.0, 0.01, -0.02), 2: w, 3: w, 4: (0.01, 0.0, 0.0), 5: w},
                    pressure={0: 1.01, 1: 0.995}, name="pressure_x_9x5x6"),
        LatticeSpec(6, 8, 5, 0.7, {0: w, 1: w, 3: (0.0, 0.03, 0.0), 4: w, 5: w}, pressure={2: 1.015},
                    name="pressure_in_velocity_out_6x8x5"),
    ]


@dataclass
class ChannelSetup:
    """A channel through the box with staircase walls of solid nodes and
    per-node inflow/outflow velocities on the z faces."""
    spec: LatticeSpec
    solid: np.ndarray      # (nz, ny, nx) uint8, 1 = solid
    face_v: dict           # face -> (ny, nx, 3) velocities of the z faces
    centre: np.ndarray     # (nz,) channel centre line x_c(z)
    half_width: float      # along x
    direction: np.ndarray  # unit vector of the channel axis
    v0: float              # centre-line speed


def tilted_channel(scale: int = 1, straight: bool = False, v0: float = 0.02, tau: float = 1.0,
                   normal_inflow: bool = False, ny: int | None = None) -> ChannelSetup:
    """The tilted channel of Sec. VI: box 64 x 8 x 128 (times `scale`), y
    periodic, channel 20 nodes wide along x (times `scale`) whose centre line
    runs from x = 11.5 at z = 0 to x = 51.5 at z = 127 (slope 40/127 for
    scale 1, the same angle for larger scales), solid nodes outside the
    channel, and the parabolic Poiseuille velocity (eq_pois) along the
    channel axis prescribed on the channel's nodes of the z = 0 and z = nz-1
    planes.  straight: the same channel along z through the box centre.
    normal_inflow: prescribe only the z component of that velocity.  ny
    overrides the periodic depth (the flow does not depend on y)."""
    nx, nz = 64 * scale, 128 * scale
    ny = 8 * scale if ny is None else int(ny)
    slope = 0.0 if straight else 40.0 / 127.0
    x0, z0 = (nx - 1) / 2.0, (nz - 1) / 2.0
    z = np.arange(nz, dtype=float)
    centre = x0 + slope * (z - z0)
    half = 10.0 * scale
    x = np.arange(nx, dtype=float)
    dist = x[None, :] - centre[:, None]               # (nz, nx)
    fluid = np.abs(dist) < half
    solid = np.broadcast_to((~fluid)[:, None, :], (nz, ny, nx)).astype(np.uint8)
    direction = np.array([slope, 0.0, 1.0]) / np.hypot(slope, 1.0)
    face_v = {}
    for face, zi in ((4, 0), (5, nz - 1)):
        prof = np.where(fluid[zi], v0 * (1.0 - (dist[zi] / half) ** 2), 0.0)  # eq_pois
        v = prof[:, None] * direction[None, :]
        if normal_inflow:
            v[:, 0] = 0.0
            v[:, 1] = 0.0
        face_v[face] = np.ascontiguousarray(np.broadcast_to(v[None, :, :], (ny, nx, 3)))
    name = ("straight" if straight else "tilted") + f"_channel_x{scale}"
    spec = LatticeSpec(nx, ny, nz, tau, {4: (0.0, 0.0, 0.0), 5: (0.0, 0.0, 0.0)}, name=name)
    return ChannelSetup(spec, np.ascontiguousarray(solid), face_v, centre, half, direction, v0)


CELL_FLUID, CELL_WALL, CELL_SOLID = 0, 1, 2


def cells_from_solid(solid: np.ndarray) -> np.ndarray:
    """Node types of a complex geometry from a solid occupancy (nz, ny, nx)
    (periodic wrap): solid nodes with a fluid node among their 26 neighbours
    are wall nodes (the wall lies on them, Sec. V; the 26-neighbourhood makes
    the corner of a box a wall node), the others solid interior."""
    solid = np.asarray(solid, bool)
    fluid_nb = np.zeros_like(solid)
    for cz in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cx in (-1, 0, 1):
                if cx or cy or cz:
                    fluid_nb |= np.roll(~solid, shift=(cz, cy, cx), axis=(0, 1, 2))
    cell = np.full(solid.shape, CELL_FLUID, np.uint8)
    cell[solid & fluid_nb] = CELL_WALL
    cell[solid & ~fluid_nb] = CELL_SOLID
    return cell


def rib_channel(nx: int = 24, ny: int = 10, nz: int = 14, rib=(8, 13, 6), tau: float = 0.9) -> tuple:
    """A channel along x (periodic) with solid slabs two nodes thick on the
    y and z sides and a rib on the bottom wall across the whole width: rib
    nodes x in [rib[0], rib[1]], z up to rib[2].  Has plane, concave-edge,
    corner, convex-edge and edge-meets-plane wall nodes.  Returns (spec,
    cell)."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = (y <= 1) | (y >= ny - 2) | (z <= 1) | (z >= nz - 2)
    solid |= (x >= rib[0]) & (x <= rib[1]) & (z <= rib[2])
    spec = LatticeSpec(nx, ny, nz, tau, {}, name=f"rib_channel_{nx}x{ny}x{nz}")
    return spec, cells_from_solid(solid)


def perturbation(shape, seed: int, amp: float) -> np.ndarray:
    """Multiplicative noise 1 + amp * U(-1, 1) of the given shape."""
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.uniform(-1.0, 1.0, shape)


def all_classes_lattices():
    """Small lattices that contain every node class (bulk, 6 faces, 12 edges,
    8 corners), mixed periodic and bounded axes, and moving walls on every
    face, for node-by-node parity."""
    out = [
        duct(5, 5, 5, (0.04, 0.01, 0.01), 0.8),
        duct(8, 7, 6, (0.03, -0.02, 0.015), 0.7),
        LatticeSpec(9, 6, 7, 1.3, {0: (0.02, 0.01, -0.01), 1: (-0.01, 0.02, 0.01), 2: (0.01, 0.03, -0.02),
                                   3: (0.02, -0.01, 0.01), 4: (-0.02, 0.01, 0.03), 5: (0.01, -0.02, -0.01)},
                    name="moving_walls_9x6x7"),
        LatticeSpec(7, 6, 5, 0.9, {2: (0.0, 0.0, 0.0), 3: (0.0, 0.0, 0.0), 4: (0.02, 0.01, 0.0),
                                   5: (-0.01, 0.0, 0.02)}, name="x_periodic_7x6x5"),
        LatticeSpec(6, 5, 8, 0.75, {0: (0.03, 0.0, 0.01), 1: (0.02, 0.01, 0.0)}, name="yz_periodic_6x5x8"),
    ]
    return out
