"""ctypes binding of the C ABI in include/lbm.h (liblbm.so, HIP for gfx950).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Functions keep the C names; a failed call raises LBMError carrying
the status code and lbm_last_error().  Device pointers may be given as ints or
as torch tensors (their data_ptr()); streams as ints, torch streams or None.

Importing this module does not need a GPU; loading the library does need the
built liblbm.so, and the module refuses to run without it (there is no
fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_ERR_ARG, LBM_ERR_OOM, LBM_ERR_HIP, LBM_ERR_STATE, LBM_ERR_NONFINITE = 0, -1, -2, -3, -4, -5
LBM_STORE_F64, LBM_STORE_F32, LBM_STORE_F16_DEV, LBM_STORE_F16_DEV_SR = 0, 1, 2, 3
LBM_X0, LBM_X1, LBM_Y0, LBM_Y1, LBM_Z0, LBM_Z1 = range(6)

STORAGE_NAMES = {LBM_STORE_F64: "f64", LBM_STORE_F32: "f32", LBM_STORE_F16_DEV: "f16dev", LBM_STORE_F16_DEV_SR: "f16sr"}

# Every symbol include/lbm.h declares.
EXPORTS = (
    "lbm_create", "lbm_create_on_buffers", "lbm_set_velocity_bc", "lbm_set_pressure_bc", "lbm_set_velocity_field",
    "lbm_set_solid_mask", "lbm_set_geometry", "lbm_classify_geometry", "lbm_set_rule_options", "lbm_set_body_force",
    "lbm_clear_bc", "lbm_step",
    "lbm_moments", "lbm_totals", "lbm_get_populations", "lbm_set_populations", "lbm_state_buffer",
    "lbm_set_layout", "lbm_get_layout", "lbm_buffer_elements",
    "lbm_element_bytes", "lbm_population_pitch", "lbm_set_launch", "lbm_get_launch", "lbm_autotune", "lbm_get_step",
    "lbm_tune_placement", "lbm_probe", "lbm_get_size", "lbm_totals_static", "lbm_set_steps_per_pass", "lbm_get_steps_per_pass",
    "lbm_destroy", "lbm_last_error",
    "lbm_job_bytes", "lbm_batch_create", "lbm_batch_submit", "lbm_batch_run_chunk", "lbm_batch_poll",
    "lbm_batch_result", "lbm_batch_set_shape", "lbm_batch_get_shape", "lbm_batch_autotune", "lbm_batch_set_policy",
    "lbm_batch_memory", "lbm_batch_set_lanes", "lbm_batch_get_stats", "lbm_batch_set_steps_per_pass",
    "lbm_batch_get_steps_per_pass", "lbm_batch_destroy",
)

LBM_JOB_QUEUED, LBM_JOB_RUNNING, LBM_JOB_DONE = 0, 1, 2
LBM_BATCH_LOCKSTEP, LBM_BATCH_SHORTEST_FIRST, LBM_BATCH_LARGE_IN_ORDER = 0, 1, 2
LBM_RULE_NO_TRANSVERSE = 1
LBM_XCD_NONE, LBM_XCD_SLABS, LBM_XCD_ROWS = 0, 1, 2  # sweep block placement on the XCDs
LBM_LAYOUT_POPULATION_MAJOR, LBM_LAYOUT_ROW_MAJOR = 0, 1  # population layout of the device buffers


class LbmJob(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
        ("storage", ctypes.c_int), ("bc_mask", ctypes.c_uint),
        ("bc_velocity", (ctypes.c_double * 3) * 6),
        ("force", ctypes.c_double * 3),
        ("u_ref", ctypes.c_double), ("tol", ctypes.c_double), ("max_steps", ctypes.c_int),
        ("pressure_mask", ctypes.c_uint), ("bc_rho", ctypes.c_double * 6),
    ]


class LbmJobStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("steps", ctypes.c_int), ("delta", ctypes.c_double),
                ("converged", ctypes.c_int), ("nodes", ctypes.c_longlong)]


class LbmBatchStats(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int), ("chunks", ctypes.c_longlong), ("job_chunks", ctypes.c_longlong),
                ("multi_job_chunks", ctypes.c_longlong), ("max_jobs_in_chunk", ctypes.c_int),
                ("overlapped_chunks", ctypes.c_longlong), ("max_lanes_running", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LBMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lbm status {status}: {message}")
        self.status = status


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def load_library(path: str = LIB_PATH):
    """Load liblbm.so (once).  Raises FileNotFoundError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_0811_4593_amd/build.py`")
    # One HIP runtime per process: when PyTorch is installed it is imported
    # first, so that liblbm.so binds to the HIP runtime torch loaded (loading
    # the system runtime first and torch's afterwards leaves two runtimes that
    # do not see each other's devices and memory).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    st = ctypes.c_int
    lib.lbm_create.argtypes = [st, st, st, ctypes.c_double, ctypes.c_double, _dp, st, _vp, ctypes.POINTER(_vp)]
    lib.lbm_create_on_buffers.argtypes = [st, st, st, ctypes.c_double, ctypes.c_double, _dp, st, _vp, _vp, _vp,
                                          ctypes.c_size_t, ctypes.POINTER(_vp)]
    lib.lbm_set_velocity_bc.argtypes = [_vp, st, _dp]
    lib.lbm_set_pressure_bc.argtypes = [_vp, st, ctypes.c_double, _dp]
    lib.lbm_set_velocity_field.argtypes = [_vp, st, _dp]
    lib.lbm_set_solid_mask.argtypes = [_vp, ctypes.POINTER(ctypes.c_ubyte)]
    lib.lbm_set_rule_options.argtypes = [_vp, ctypes.c_uint]
    lib.lbm_set_geometry.argtypes = [_vp, ctypes.POINTER(ctypes.c_ubyte)]
    lib.lbm_classify_geometry.argtypes = [st, st, st, ctypes.POINTER(ctypes.c_ubyte), ctypes.POINTER(ctypes.c_uint),
                                          ctypes.POINTER(ctypes.c_longlong)]
    lib.lbm_set_body_force.argtypes = [_vp, _dp]
    lib.lbm_clear_bc.argtypes = [_vp, st]
    lib.lbm_step.argtypes = [_vp, st]
    lib.lbm_moments.argtypes = [_vp, _vp, _vp, st]
    lib.lbm_totals.argtypes = [_vp, _dp, _dp]
    lib.lbm_get_populations.argtypes = [_vp, _dp]
    lib.lbm_set_populations.argtypes = [_vp, _dp]
    lib.lbm_state_buffer.argtypes = [_vp, ctypes.POINTER(_vp)]
    lib.lbm_set_layout.argtypes = [_vp, st]
    lib.lbm_get_layout.argtypes = [_vp, ctypes.POINTER(st)]
    lib.lbm_buffer_elements.argtypes = [st, st, st, st, st]
    lib.lbm_buffer_elements.restype = ctypes.c_size_t
    lib.lbm_element_bytes.argtypes = [st]
    lib.lbm_element_bytes.restype = ctypes.c_size_t
    lib.lbm_population_pitch.argtypes = [ctypes.c_size_t]
    lib.lbm_population_pitch.restype = ctypes.c_size_t
    lib.lbm_set_launch.argtypes = [_vp, st, st, st]
    lib.lbm_get_launch.argtypes = [_vp, ctypes.POINTER(st), ctypes.POINTER(st), ctypes.POINTER(st)]
    lib.lbm_autotune.argtypes = [_vp, st, ctypes.POINTER(st), ctypes.POINTER(st), ctypes.POINTER(st)]
    lib.lbm_get_step.argtypes = [_vp, ctypes.POINTER(ctypes.c_ulonglong)]
    lib.lbm_tune_placement.argtypes = [_vp, st, st, ctypes.POINTER(st), _dp, _dp]
    lib.lbm_probe.argtypes = [_vp, st, st]
    lib.lbm_get_size.argtypes = [_vp, ctypes.POINTER(st), ctypes.POINTER(st), ctypes.POINTER(st)]
    lib.lbm_set_steps_per_pass.argtypes = [_vp, st, st, st]
    lib.lbm_get_steps_per_pass.argtypes = [_vp, ctypes.POINTER(st), ctypes.POINTER(st), ctypes.POINTER(st)]
    lib.lbm_destroy.argtypes = [_vp]
    lib.lbm_destroy.restype = None
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = ctypes.c_char_p
    ip = ctypes.POINTER(ctypes.c_int)
    szp = ctypes.POINTER(ctypes.c_size_t)
    lib.lbm_job_bytes.argtypes = [ctypes.POINTER(LbmJob), szp]
    lib.lbm_batch_create.argtypes = [ctypes.c_size_t, st, st, _vp, ctypes.POINTER(_vp)]
    lib.lbm_batch_submit.argtypes = [_vp, ctypes.POINTER(LbmJob), ip]
    lib.lbm_batch_run_chunk.argtypes = [_vp, ip, ip]
    lib.lbm_batch_poll.argtypes = [_vp, st, ctypes.POINTER(LbmJobStatus)]
    lib.lbm_batch_result.argtypes = [_vp, st, _vp, _vp]
    lib.lbm_batch_set_shape.argtypes = [_vp, st, st, st]
    lib.lbm_batch_set_policy.argtypes = [_vp, st, ctypes.c_size_t]
    lib.lbm_batch_get_shape.argtypes = [_vp, ip, ip, ip]
    lib.lbm_batch_autotune.argtypes = [_vp, st, ip, ip, ip]
    lib.lbm_batch_memory.argtypes = [_vp, szp, szp]
    lib.lbm_batch_set_lanes.argtypes = [_vp, st]
    lib.lbm_batch_set_steps_per_pass.argtypes = [_vp, st, st]
    lib.lbm_batch_get_steps_per_pass.argtypes = [_vp, ctypes.POINTER(st), ctypes.POINTER(st)]
    lib.lbm_batch_get_stats.argtypes = [_vp, ctypes.POINTER(LbmBatchStats)]
    lib.lbm_batch_destroy.argtypes = [_vp]
    lib.lbm_batch_destroy.restype = None
    for name in EXPORTS:
        if name not in ("lbm_element_bytes", "lbm_population_pitch", "lbm_buffer_elements", "lbm_destroy",
                        "lbm_last_error",
                        "lbm_batch_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != LBM_OK:
        raise LBMError(status, lbm_last_error())


def _dev(p) -> int | None:
    if p is None:
        return None
    if hasattr(p, "data_ptr"):
        return int(p.data_ptr())
    return int(p)


def _stream(s) -> int | None:
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream)
    return int(s)


def _vec3(u) -> ctypes.Array:
    a = (ctypes.c_double * 3)()
    for i, x in enumerate(u):
        a[i] = float(x)
    return a


def _host_array(a, dtype, count: int, what: str, writable: bool = False):
    """A C-contiguous host array of `count` elements of `dtype` for a C call;
    raises ValueError when the size does not match (the C side reads or
    writes exactly `count` elements)."""
    if writable:
        if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags["C_CONTIGUOUS"] \
                or not a.flags["WRITEABLE"]:
            raise ValueError(f"{what} must be a writable C-contiguous {np.dtype(dtype).name} numpy array")
    else:
        a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if a.size != count:
        raise ValueError(f"{what} has {a.size} elements; {count} expected")
    return a


def _node_types(cell, count: int, what: str):
    """Node types 0, 1, 2 as uint8, checked before any conversion (a cast
    would turn 256 into 0 or 0.5 into 0)."""
    c = np.asarray(cell)
    if c.size != count:
        raise ValueError(f"{what} has {c.size} entries; {count} expected")
    if c.dtype.kind not in "biu":
        raise ValueError(f"{what} must hold integers 0, 1 or 2 (got dtype {c.dtype})")
    if c.size and (c.min() < 0 or c.max() > 2):
        raise ValueError(f"{what} must hold integers 0, 1 or 2 (found {c.min()}..{c.max()})")
    return np.ascontiguousarray(c.astype(np.uint8))


def lbm_get_size(h):
    nx, ny, nz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_get_size(h, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(nz)))
    return nx.value, ny.value, nz.value


def _nodes(h) -> int:
    nx, ny, nz = lbm_get_size(h)
    return nx * ny * nz


def lbm_last_error() -> str:
    return load_library().lbm_last_error().decode()


def lbm_element_bytes(storage: int) -> int:
    return int(load_library().lbm_element_bytes(int(storage)))


def lbm_population_pitch(nodes: int) -> int:
    return int(load_library().lbm_population_pitch(int(nodes)))


def lbm_create(nx, ny, nz, tau, rho0=1.0, u0=(0.0, 0.0, 0.0), storage=LBM_STORE_F32, stream=None) -> int:
    h = _vp()
    _check(load_library().lbm_create(int(nx), int(ny), int(nz), float(tau), float(rho0),
                                     None if u0 is None else _vec3(u0), int(storage), _stream(stream),
                                     ctypes.byref(h)))
    return h.value


def lbm_create_on_buffers(nx, ny, nz, tau, rho0, u0, storage, stream, buf_a, buf_b, buf_bytes) -> int:
    h = _vp()
    _check(load_library().lbm_create_on_buffers(int(nx), int(ny), int(nz), float(tau), float(rho0),
                                                None if u0 is None else _vec3(u0), int(storage),
                                                _stream(stream), _dev(buf_a), _dev(buf_b), int(buf_bytes),
                                                ctypes.byref(h)))
    return h.value


def lbm_set_velocity_bc(h, face, u):
    _check(load_library().lbm_set_velocity_bc(h, int(face), _vec3(u)))


def lbm_set_pressure_bc(h, face, rho0, u_t=None):
    _check(load_library().lbm_set_pressure_bc(h, int(face), float(rho0), None if u_t is None else _vec3(u_t)))


def lbm_set_velocity_field(h, face, v=None):
    """v: per-node velocities of the face, float64 array of 3 * n_face values
    (e.g. shape (n2, n1, 3) over the face's two other axes), or None."""
    if v is None:
        _check(load_library().lbm_set_velocity_field(h, int(face), None))
        return
    nx, ny, nz = lbm_get_size(h)
    if not 0 <= int(face) <= 5:
        raise ValueError(f"invalid face {face}")
    n_face = (ny * nz, nx * nz, nx * ny)[int(face) // 2]
    a = _host_array(v, np.float64, 3 * n_face, "face velocity field")
    _check(load_library().lbm_set_velocity_field(h, int(face), a.ctypes.data_as(_dp)))


def lbm_set_solid_mask(h, solid=None):
    """solid: (nz, ny, nx) array, non-zero = solid node; None removes it."""
    if solid is None:
        _check(load_library().lbm_set_solid_mask(h, None))
        return
    a = np.asarray(solid)
    if a.size != _nodes(h):
        raise ValueError(f"solid mask has {a.size} entries; {_nodes(h)} expected")
    a = np.ascontiguousarray(a != 0).astype(np.uint8)  # any non-zero value is solid
    _check(load_library().lbm_set_solid_mask(h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))))


def lbm_set_geometry(h, cell=None):
    """cell: (nz, ny, nx) node types (0 fluid, 1 wall, 2 solid interior), or None."""
    if cell is None:
        _check(load_library().lbm_set_geometry(h, None))
        return
    a = _node_types(cell, _nodes(h), "geometry")
    _check(load_library().lbm_set_geometry(h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))))


GEO_FLUID, GEO_SOLID, GEO_PLANE_EDGE_CORNER, GEO_CONVEX_EDGE, GEO_GENERAL = range(5)


def lbm_classify_geometry(cell):
    """Host-only classification of (nz, ny, nx) node types; returns (code
    array of the same shape, uint32; counts per kind)."""
    nz, ny, nx = np.asarray(cell).shape
    a = _node_types(cell, nx * ny * nz, "geometry")
    code = np.zeros(a.shape, np.uint32)
    counts = (ctypes.c_longlong * 5)()
    _check(load_library().lbm_classify_geometry(nx, ny, nz, a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                                                code.ctypes.data_as(ctypes.POINTER(ctypes.c_uint)), counts))
    return code, list(counts)


def lbm_set_rule_options(h, flags: int):
    _check(load_library().lbm_set_rule_options(h, int(flags)))


def lbm_set_body_force(h, F):
    _check(load_library().lbm_set_body_force(h, _vec3(F)))


def lbm_clear_bc(h, face):
    _check(load_library().lbm_clear_bc(h, int(face)))


def lbm_step(h, nsteps: int = 1):
    _check(load_library().lbm_step(h, int(nsteps)))


def lbm_moments(h, rho=None, u=None, dst_on_device: bool = False):
    """Host mode: rho (N,) and u (3*N,) float64 numpy arrays (C-contiguous)
    are filled.  Device mode: rho/u are device pointers or torch tensors."""
    if dst_on_device:
        _check(load_library().lbm_moments(h, _dev(rho), _dev(u), 1))
        return
    n = _nodes(h)
    if rho is not None:
        _host_array(rho, np.float64, n, "rho", writable=True)
    if u is not None:
        _host_array(u, np.float64, 3 * n, "u", writable=True)
    _check(load_library().lbm_moments(h, None if rho is None else rho.ctypes.data,
                                      None if u is None else u.ctypes.data, 0))


def lbm_totals(h):
    m = ctypes.c_double()
    j = (ctypes.c_double * 3)()
    _check(load_library().lbm_totals(h, ctypes.byref(m), j))
    return m.value, np.array(list(j))


def lbm_get_populations(h, out: np.ndarray):
    _host_array(out, np.float64, 19 * _nodes(h), "populations", writable=True)
    _check(load_library().lbm_get_populations(h, out.ctypes.data_as(_dp)))
    return out


def lbm_set_populations(h, f: np.ndarray):
    f = _host_array(f, np.float64, 19 * _nodes(h), "populations")
    _check(load_library().lbm_set_populations(h, f.ctypes.data_as(_dp)))


def lbm_state_buffer(h) -> int:
    p = _vp()
    _check(load_library().lbm_state_buffer(h, ctypes.byref(p)))
    return p.value


def lbm_set_layout(h, layout: int):
    _check(load_library().lbm_set_layout(h, int(layout)))


def lbm_buffer_elements(nx: int, ny: int, nz: int, storage: int, layout: int) -> int:
    return int(load_library().lbm_buffer_elements(int(nx), int(ny), int(nz), int(storage), int(layout)))


def lbm_get_layout(h) -> int:
    v = ctypes.c_int()
    _check(load_library().lbm_get_layout(h, ctypes.byref(v)))
    return v.value


def lbm_set_launch(h, block_x: int, nodes_per_thread: int, xcd_remap: int):
    _check(load_library().lbm_set_launch(h, int(block_x), int(nodes_per_thread), int(xcd_remap)))


def lbm_get_launch(h):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_get_launch(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def lbm_autotune(h, trial_steps: int = 2):
    """Time the candidate launch shapes on real steps and keep the fastest;
    returns (block_x, nodes_per_thread, xcd_remap)."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_autotune(h, int(trial_steps), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def lbm_tune_placement(h, max_buffers: int = 6, trial_steps: int = 1):
    """Time the lattice's state on every pair of a pool of up to max_buffers
    device buffers (real steps) and keep the fastest pair; returns
    (buffers_tried, ms_per_step_before, ms_per_step_after)."""
    n = ctypes.c_int()
    before, after = ctypes.c_double(), ctypes.c_double()
    _check(load_library().lbm_tune_placement(h, int(max_buffers), int(trial_steps), ctypes.byref(n),
                                             ctypes.byref(before), ctypes.byref(after)))
    return n.value, before.value, after.value


def lbm_set_steps_per_pass(h, steps_per_pass: int, z_planes: int = 0, tile_rows: int = 0):
    _check(load_library().lbm_set_steps_per_pass(h, int(steps_per_pass), int(z_planes), int(tile_rows)))


def lbm_get_steps_per_pass(h):
    """(steps_per_pass, z_planes, tile_rows)"""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_get_steps_per_pass(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def lbm_get_step(h) -> int:
    s = ctypes.c_ulonglong()
    _check(load_library().lbm_get_step(h, ctypes.byref(s)))
    return s.value


def lbm_probe(h, kind: int, nrep: int = 1):
    _check(load_library().lbm_probe(h, int(kind), int(nrep)))


def lbm_destroy(h):
    if h:
        load_library().lbm_destroy(h)


def make_job(nx, ny, nz, tau, bc, storage=LBM_STORE_F32, rho0=1.0, u_ref=None, tol=0.0, max_steps=0,
             force=(0.0, 0.0, 0.0), pressure=None) -> LbmJob:
    """An lbm_job from a face -> velocity mapping and a face -> density
    mapping of pressure faces (whose velocity in `bc`, if any, is the
    tangential velocity); u_ref defaults to the largest prescribed speed (or
    1 when every face is at rest)."""
    j = LbmJob()
    j.nx, j.ny, j.nz = int(nx), int(ny), int(nz)
    j.tau, j.rho0, j.storage = float(tau), float(rho0), int(storage)
    mask = 0
    vmax = 0.0
    for face, v in bc.items():
        mask |= 1 << int(face)
        for a in range(3):
            j.bc_velocity[int(face)][a] = float(v[a])
        vmax = max(vmax, float(np.linalg.norm(np.asarray(v, dtype=float))))
    pmask = 0
    for face, r in (pressure or {}).items():
        mask |= 1 << int(face)
        pmask |= 1 << int(face)
        j.bc_rho[int(face)] = float(r)
    j.bc_mask = mask
    j.pressure_mask = pmask
    for a in range(3):
        j.force[a] = float(force[a])
    j.u_ref = float(u_ref) if u_ref is not None else (vmax if vmax > 0 else 1.0)
    j.tol, j.max_steps = float(tol), int(max_steps)
    return j


def lbm_job_bytes(job: LbmJob) -> int:
    b = ctypes.c_size_t()
    _check(load_library().lbm_job_bytes(ctypes.byref(job), ctypes.byref(b)))
    return b.value


def lbm_batch_create(hbm_budget_bytes: int, chunk_steps: int = 100, max_jobs: int = 1024, stream=None) -> int:
    h = _vp()
    _check(load_library().lbm_batch_create(int(hbm_budget_bytes), int(chunk_steps), int(max_jobs),
                                           _stream(stream), ctypes.byref(h)))
    return h.value


def lbm_batch_submit(b, job: LbmJob) -> int:
    i = ctypes.c_int()
    _check(load_library().lbm_batch_submit(b, ctypes.byref(job), ctypes.byref(i)))
    return i.value


def lbm_batch_run_chunk(b):
    a, q = ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_batch_run_chunk(b, ctypes.byref(a), ctypes.byref(q)))
    return a.value, q.value


def lbm_batch_poll(b, job_id: int) -> LbmJobStatus:
    st = LbmJobStatus()
    _check(load_library().lbm_batch_poll(b, int(job_id), ctypes.byref(st)))
    return st


def lbm_batch_result(b, job_id: int, nodes):
    """(rho, u) of a finished job, then the job is forgotten; nodes=None
    forgets it without copying and returns (None, None).  nodes must be the
    job's node count."""
    if nodes is None:
        _check(load_library().lbm_batch_result(b, int(job_id), None, None))
        return None, None
    have = lbm_batch_poll(b, job_id).nodes
    if int(nodes) != have:
        raise ValueError(f"job {job_id} has {have} nodes, not {nodes}")
    rho = np.empty(have)
    u = np.empty(3 * have)
    _check(load_library().lbm_batch_result(b, int(job_id), rho.ctypes.data, u.ctypes.data))
    return rho, u


def lbm_batch_set_shape(b, block_x: int, tile_nodes: int, grid_blocks: int = 0):
    _check(load_library().lbm_batch_set_shape(b, int(block_x), int(tile_nodes), int(grid_blocks)))


def lbm_batch_set_policy(b, policy: int, fill_nodes: int = 0):
    _check(load_library().lbm_batch_set_policy(b, int(policy), int(fill_nodes)))


def lbm_batch_get_shape(b):
    x, t, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_batch_get_shape(b, ctypes.byref(x), ctypes.byref(t), ctypes.byref(g)))
    return x.value, t.value, g.value


def lbm_batch_autotune(b, trial_steps: int = 4):
    x, t, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_batch_autotune(b, int(trial_steps), ctypes.byref(x), ctypes.byref(t),
                                             ctypes.byref(g)))
    return x.value, t.value, g.value


def lbm_batch_memory(b):
    u, c = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().lbm_batch_memory(b, ctypes.byref(u), ctypes.byref(c)))
    return u.value, c.value


def lbm_batch_set_lanes(b, lanes: int):
    _check(load_library().lbm_batch_set_lanes(b, int(lanes)))


def lbm_batch_set_steps_per_pass(b, steps_per_pass: int, z_planes: int = 0):
    """1 (the default): one step per launch; 2: passes of two steps over
    every job (row-major jobs; set before submitting)."""
    _check(load_library().lbm_batch_set_steps_per_pass(b, int(steps_per_pass), int(z_planes)))


def lbm_batch_get_steps_per_pass(b):
    sp, zc = ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_batch_get_steps_per_pass(b, ctypes.byref(sp), ctypes.byref(zc)))
    return sp.value, zc.value


def lbm_batch_get_stats(b) -> dict:
    st = LbmBatchStats()
    _check(load_library().lbm_batch_get_stats(b, ctypes.byref(st)))
    return st.as_dict()


def lbm_batch_destroy(b):
    if b:
        load_library().lbm_batch_destroy(b)


class Lattice:
    """Owning wrapper of one lbm_lattice handle (convenience only)."""

    def __init__(self, nx, ny, nz, tau, rho0=1.0, u0=(0.0, 0.0, 0.0), storage=LBM_STORE_F32, stream=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.storage = int(storage)
        self.h = lbm_create(nx, ny, nz, tau, rho0, u0, storage, stream)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (19, self.nz, self.ny, self.nx)

    def set_velocity_bc(self, face, u):
        lbm_set_velocity_bc(self.h, face, u)

    def step(self, n=1):
        lbm_step(self.h, n)

    def moments(self):
        n = self.nodes
        rho = np.empty(n)
        u = np.empty(3 * n)
        lbm_moments(self.h, rho, u)
        return rho.reshape(self.nz, self.ny, self.nx), u.reshape(3, self.nz, self.ny, self.nx)

    def totals(self):
        return lbm_totals(self.h)

    def get(self) -> np.ndarray:
        out = np.empty(self.shape)
        return lbm_get_populations(self.h, out)

    def set(self, f):
        lbm_set_populations(self.h, np.asarray(f).reshape(self.shape))

    def close(self):
        lbm_destroy(self.h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.close()
        except Exception:
            pass
