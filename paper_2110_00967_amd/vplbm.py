"""ctypes binding of libvplbm.so (the C ABI in include/vplbm.h).

Argument marshalling only: every step of the VP-LBM path runs in the HIP
kernels of the library.  PyTorch supplies device memory (a uint8 tensor of
``vplbm_required_bytes``) and the current HIP stream; nothing else.

The library must have been built (``paper_2110_00967_amd/build.py``); there
is no fallback -- loading fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VPLBM_LIBRARY") or os.path.join(HERE, "libvplbm.so")

F64, F32, F16DEV = 0, 1, 2
PRECISIONS = {"f64": F64, "f32": F32, "f16dev": F16DEV}
PERIODIC, VELOCITY, FREESLIP, OUTFLOW, CONVECTIVE = 0, 1, 2, 3, 4
FORCE_ME, FORCE_SI = 0, 1
STEP_MACRO = 1
STREAM_AB, STREAM_AA = 0, 1

OK, EINVAL, ENOMEM, EHIP, ESTATE, EUNSTABLE, ENOSAMPLE = 0, -1, -2, -3, -4, -5, -6
_ERRNAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", ESTATE: "ESTATE", EUNSTABLE: "EUNSTABLE",
             ENOSAMPLE: "ENOSAMPLE"}

# every entry point of include/vplbm.h
EXPORTS = [
    "vplbm_required_bytes", "vplbm_create", "vplbm_destroy", "vplbm_last_error", "vplbm_init_uniform",
    "vplbm_set_fields", "vplbm_set_body_force", "vplbm_set_body_disk", "vplbm_set_body_polygon",
    "vplbm_set_mask", "vplbm_set_body_motion", "vplbm_set_body_dynamics", "vplbm_set_si_points",
    "vplbm_step", "vplbm_step_timed", "vplbm_sync", "vplbm_step_count", "vplbm_set_tile",
    "vplbm_get_tile", "vplbm_forces_me", "vplbm_forces_si",
    "vplbm_forces_si_at", "vplbm_force_history", "vplbm_get_body_state", "vplbm_read_macro",
    "vplbm_read_populations", "vplbm_read_mask", "vplbm_read_macro_window", "vplbm_read_populations_window",
    "vplbm_batch_create", "vplbm_batch_destroy", "vplbm_batch_last_error", "vplbm_batch_step",
    "vplbm_set_body_ids", "vplbm_set_si_points_body", "vplbm_forces_body", "vplbm_force_history_body",
    "vplbm_read_macro_device", "vplbm_batch_set_tile", "vplbm_batch_get_tile", "vplbm_batch_set_lattices",
    "vplbm_batch_step_noalloc", "vplbm_set_moving_disks", "vplbm_get_body_state_of",
]


class VplbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Edge(C.Structure):
    _fields_ = [("kind", C.c_int), ("ux", C.c_double), ("uy", C.c_double)]


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("tau", C.c_double), ("eta", C.c_double),
                ("rho0", C.c_double), ("precision", C.c_int), ("west", Edge), ("east", Edge),
                ("south", Edge), ("north", Edge), ("hist_capacity", C.c_int),
                ("max_si_points", C.c_int), ("max_vertices", C.c_int), ("trt_lambda", C.c_double),
                ("si_rule", C.c_int), ("max_bodies", C.c_int), ("max_interface_cells", C.c_int),
                ("streaming", C.c_int)]


class BodyState(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("theta", C.c_double), ("u", C.c_double),
                ("v", C.c_double), ("omega", C.c_double)]


class Disk(C.Structure):
    """One of several moving disks: rho_s > 0 free, rho_s = 0 prescribed."""
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("r", C.c_double), ("theta", C.c_double),
                ("u", C.c_double), ("v", C.c_double), ("omega", C.c_double), ("rho_s", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libvplbm.so and declare the C signatures (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run paper_2110_00967_amd/build.py)")
    # torch ships its own HIP runtime under the same soname as the system's:
    # load it first so libvplbm.so binds to that one runtime (loading ours
    # first would put two HIP/HSA runtimes in the process)
    import torch  # noqa: F401
    L = C.CDLL(path)
    P = C.POINTER
    vp, dp, ip = C.c_void_p, P(C.c_double), C.c_int
    L.vplbm_required_bytes.argtypes = [P(Params)]
    L.vplbm_required_bytes.restype = C.c_size_t
    L.vplbm_create.argtypes = [P(Params), vp, C.c_size_t, vp, P(vp)]
    L.vplbm_destroy.argtypes = [vp]
    L.vplbm_last_error.argtypes = [vp]
    L.vplbm_last_error.restype = C.c_char_p
    L.vplbm_init_uniform.argtypes = [vp, C.c_double, C.c_double, C.c_double]
    L.vplbm_set_fields.argtypes = [vp, dp, dp, dp]
    L.vplbm_set_body_force.argtypes = [vp, C.c_double, C.c_double]
    L.vplbm_set_body_disk.argtypes = [vp, C.c_double, C.c_double, C.c_double]
    L.vplbm_set_body_polygon.argtypes = [vp, dp, ip, C.c_double, C.c_double]
    L.vplbm_set_mask.argtypes = [vp, P(C.c_uint8)]
    L.vplbm_set_body_motion.argtypes = [vp, P(BodyState)]
    L.vplbm_set_body_dynamics.argtypes = [vp, C.c_double, C.c_double, C.c_double, ip]
    L.vplbm_set_si_points.argtypes = [vp, dp, dp, dp, ip]
    L.vplbm_set_si_points_body.argtypes = [vp, ip, dp, dp, dp, ip]
    L.vplbm_set_body_ids.argtypes = [vp, P(C.c_uint8), ip, dp]
    L.vplbm_forces_body.argtypes = [vp, ip, ip, dp]
    L.vplbm_force_history_body.argtypes = [vp, ip, ip, C.c_longlong, ip, dp]
    L.vplbm_step.argtypes = [vp, ip, ip]
    L.vplbm_step_timed.argtypes = [vp, ip, ip, dp]
    L.vplbm_sync.argtypes = [vp]
    L.vplbm_step_count.argtypes = [vp]
    L.vplbm_step_count.restype = C.c_longlong
    L.vplbm_set_tile.argtypes = [vp, ip, ip]
    L.vplbm_get_tile.argtypes = [vp, P(C.c_int), P(C.c_int)]
    L.vplbm_forces_me.argtypes = [vp, dp]
    L.vplbm_forces_si.argtypes = [vp, dp]
    L.vplbm_forces_si_at.argtypes = [vp, dp, dp, dp, ip, dp]
    L.vplbm_force_history.argtypes = [vp, ip, C.c_longlong, ip, dp]
    L.vplbm_get_body_state.argtypes = [vp, P(BodyState)]
    L.vplbm_get_body_state_of.argtypes = [vp, ip, P(BodyState)]
    L.vplbm_set_moving_disks.argtypes = [vp, P(Disk), ip, C.c_double, C.c_double, ip]
    L.vplbm_read_macro.argtypes = [vp, dp, dp, dp]
    L.vplbm_read_populations.argtypes = [vp, dp]
    L.vplbm_read_macro_window.argtypes = [vp, ip, ip, ip, ip, dp, dp, dp]
    L.vplbm_read_populations_window.argtypes = [vp, ip, ip, ip, ip, dp]
    L.vplbm_read_mask.argtypes = [vp, P(C.c_uint8)]
    L.vplbm_batch_create.argtypes = [P(vp), ip, P(vp)]
    L.vplbm_batch_destroy.argtypes = [vp]
    L.vplbm_batch_last_error.argtypes = [vp]
    L.vplbm_batch_last_error.restype = C.c_char_p
    L.vplbm_batch_step.argtypes = [vp, P(C.c_int)]
    L.vplbm_batch_set_tile.argtypes = [vp, ip, ip]
    L.vplbm_batch_set_lattices.argtypes = [vp, P(vp), ip]
    L.vplbm_batch_get_tile.argtypes = [vp, P(C.c_int), P(C.c_int)]
    L.vplbm_batch_step_noalloc.argtypes = [P(vp), ip, P(C.c_int)]
    for name in EXPORTS:
        if name not in ("vplbm_required_bytes", "vplbm_last_error", "vplbm_step_count", "vplbm_batch_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def make_params(nx, ny, tau, eta, rho0=1.0, precision="f32", west=(PERIODIC, 0, 0), east=(PERIODIC, 0, 0),
                south=(PERIODIC, 0, 0), north=(PERIODIC, 0, 0), hist_capacity=0, max_si_points=0,
                max_vertices=0, trt_lambda=0.0, si_rule=0, max_bodies=0, max_interface_cells=0,
                streaming=0) -> Params:
    p = Params()
    p.nx, p.ny, p.tau, p.eta, p.rho0 = int(nx), int(ny), float(tau), float(eta), float(rho0)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for name, e in (("west", west), ("east", east), ("south", south), ("north", north)):
        setattr(p, name, Edge(int(e[0]), float(e[1]), float(e[2])))
    p.hist_capacity, p.max_si_points, p.max_vertices = hist_capacity, max_si_points, max_vertices
    p.trt_lambda = float(trt_lambda)
    p.si_rule = int(si_rule)
    p.max_bodies = int(max_bodies)
    p.max_interface_cells = int(max_interface_cells)
    p.streaming = int(streaming)
    return p


def required_bytes(params: Params) -> int:
    return int(load_library().vplbm_required_bytes(C.byref(params)))


def case_params(case, precision="f32", **kw) -> Params:
    """Parameters of a workload description (grid, relaxation, edges, point
    and vertex capacities, collision, stencil rule); kw adds any other
    make_params argument.  Lattice.from_case creates its lattice from them,
    so required_bytes(case_params(...)) is that lattice's device size."""
    e = lambda E: (E.kind, E.ux, E.uy)
    npts = 0 if case.si_xy is None else len(case.si_xy)
    nv = 0 if case.polygon is None else len(case.polygon)
    return make_params(case.nx, case.ny, case.tau, case.eta, case.rho0, precision, e(case.west), e(case.east),
                       e(case.south), e(case.north), max_si_points=max(npts, 16), max_vertices=max(nv, 16),
                       trt_lambda=getattr(case, "trt_lambda", 0.0), si_rule=getattr(case, "si_rule", 0), **kw)


class Lattice:
    """One VP-LBM lattice on the current GPU, memory from a torch tensor."""

    def __init__(self, params: Params, stream=None, device_buffer=None):
        import torch  # device memory and the stream only

        self._lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the VP-LBM library runs on the device only")
        self.params = params
        self.nx, self.ny = params.nx, params.ny
        nbytes = required_bytes(params)
        if nbytes == 0:
            raise VplbmError(EINVAL, "invalid lattice parameters")
        if device_buffer is None:
            device_buffer = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._buf = device_buffer
        self.nbytes = nbytes
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = C.c_void_p()
        rc = self._lib.vplbm_create(C.byref(params), C.c_void_p(device_buffer.data_ptr()),
                                    C.c_size_t(device_buffer.numel()), C.c_void_p(stream.cuda_stream),
                                    C.byref(h))
        if rc != OK:
            why = self._lib.vplbm_last_error(None).decode(errors="replace")
            raise VplbmError(rc, f"vplbm_create failed: {why}")
        self._h = h

    @classmethod
    def from_case(cls, case, precision="f32", **kw):
        lat = cls(case_params(case, precision, **kw))
        if case.gx or case.gy:
            lat.set_body_force(case.gx, case.gy)
        if case.disk is not None:
            lat.set_disk(*case.disk)
        elif case.polygon is not None:
            lat.set_polygon(case.polygon, case.ref_point)
        if case.si_xy is not None:
            lat.set_si_points(case.si_xy, case.si_n, case.si_ds)
        if case.rho_s is not None:
            lat.set_dynamics(case.rho_s, case.grav[0], case.grav[1], case.force_source)
        lat.init_uniform(case.rho0, *case.u_init)
        return lat

    # -- plumbing -----------------------------------------------------------
    def _chk(self, rc):
        if rc != OK:
            msg = self._lib.vplbm_last_error(self._h).decode(errors="replace")
            raise VplbmError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.vplbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup --------------------------------------------------------------
    def init_uniform(self, rho=1.0, ux=0.0, uy=0.0):
        self._chk(self._lib.vplbm_init_uniform(self._h, rho, ux, uy))

    def set_fields(self, rho, ux, uy):
        shp = (self.ny, self.nx)
        r, a, b = _f64(rho, shp), _f64(ux, shp), _f64(uy, shp)
        self._chk(self._lib.vplbm_set_fields(self._h, _dptr(r), _dptr(a), _dptr(b)))

    def set_body_force(self, gx, gy):
        self._chk(self._lib.vplbm_set_body_force(self._h, gx, gy))

    def set_disk(self, xc, yc, r):
        self._chk(self._lib.vplbm_set_body_disk(self._h, xc, yc, r))

    def set_polygon(self, xy, ref):
        v = _f64(xy)
        self._chk(self._lib.vplbm_set_body_polygon(self._h, _dptr(v), len(v), ref[0], ref[1]))

    def set_mask(self, solid):
        m = np.ascontiguousarray((np.asarray(solid) != 0).astype(np.uint8).reshape(self.ny, self.nx))
        self._chk(self._lib.vplbm_set_mask(self._h, m.ctypes.data_as(C.POINTER(C.c_uint8))))

    def set_body_ids(self, ids, refs):
        """Several static bodies: ids [ny][nx] (0 fluid, 1..nbody) and each body's reference point."""
        m = np.ascontiguousarray(np.asarray(ids, dtype=np.uint8).reshape(self.ny, self.nx))
        r = _f64(refs).reshape(-1, 2)
        self._chk(self._lib.vplbm_set_body_ids(self._h, m.ctypes.data_as(C.POINTER(C.c_uint8)), len(r),
                                               _dptr(np.ascontiguousarray(r))))

    def set_si_points_body(self, body, xy, nrm, ds):
        xy, nrm, ds = _f64(xy), _f64(nrm), _f64(ds)
        self._chk(self._lib.vplbm_set_si_points_body(self._h, int(body), _dptr(xy), _dptr(nrm), _dptr(ds),
                                                     len(ds)))

    def set_motion(self, x, y, theta, u, v, omega):
        s = BodyState(x, y, theta, u, v, omega)
        self._chk(self._lib.vplbm_set_body_motion(self._h, C.byref(s)))

    def set_moving_disks(self, disks, gx=0.0, gy=0.0, source=FORCE_ME):
        """Several moving disks, each (x, y, r, theta, u, v, omega, rho_s); rho_s = 0: prescribed."""
        arr = (Disk * len(disks))(*[Disk(*[float(v) for v in d]) for d in disks])
        self._chk(self._lib.vplbm_set_moving_disks(self._h, arr, len(disks), gx, gy, int(source)))

    def set_dynamics(self, rho_s, gx, gy, source=FORCE_ME):
        self._chk(self._lib.vplbm_set_body_dynamics(self._h, rho_s, gx, gy, int(source)))

    def set_si_points(self, xy, nrm, ds):
        xy, nrm, ds = _f64(xy), _f64(nrm), _f64(ds)
        n = len(ds)
        self._chk(self._lib.vplbm_set_si_points(self._h, _dptr(xy), _dptr(nrm), _dptr(ds), n))

    # -- time stepping -------------------------------------------------------
    def step(self, n=1, macro=False):
        self._chk(self._lib.vplbm_step(self._h, int(n), STEP_MACRO if macro else 0))

    def step_timed(self, n=1, macro=False):
        """Step like step(); returns the summed step-kernel time in ms (HIP events)."""
        ms = np.zeros(1)
        self._chk(self._lib.vplbm_step_timed(self._h, int(n), STEP_MACRO if macro else 0, _dptr(ms)))
        return float(ms[0])

    def sync(self):
        self._chk(self._lib.vplbm_sync(self._h))

    def set_tile(self, bx, by):
        self._chk(self._lib.vplbm_set_tile(self._h, int(bx), int(by)))

    @property
    def tile(self):
        """(bx, by): the step tile this lattice's own steps use."""
        bx, by = C.c_int(0), C.c_int(0)
        self._chk(self._lib.vplbm_get_tile(self._h, C.byref(bx), C.byref(by)))
        return bx.value, by.value

    @property
    def step_count(self):
        return int(self._lib.vplbm_step_count(self._h))

    # -- results ------------------------------------------------------------
    def forces_me(self):
        o = np.zeros(3)
        self._chk(self._lib.vplbm_forces_me(self._h, _dptr(o)))
        return o

    def forces_si(self):
        o = np.zeros(3)
        self._chk(self._lib.vplbm_forces_si(self._h, _dptr(o)))
        return o

    def forces_si_at(self, xy, nrm, ds):
        xy, nrm, ds = _f64(xy), _f64(nrm), _f64(ds)
        o = np.zeros(3)
        self._chk(self._lib.vplbm_forces_si_at(self._h, _dptr(xy), _dptr(nrm), _dptr(ds), len(ds), _dptr(o)))
        return o

    def forces_body(self, body, which):
        o = np.zeros(3)
        self._chk(self._lib.vplbm_forces_body(self._h, int(body), int(which), _dptr(o)))
        return o

    def force_history(self, which, first, n, body=1):
        o = np.zeros((n, 3))
        self._chk(self._lib.vplbm_force_history_body(self._h, int(body), int(which), int(first), int(n), _dptr(o)))
        return o

    def history(self, which, body=1):
        """All kept forces of steps 1..step_count (up to the ring capacity)."""
        n = self.step_count
        cap = self.params.hist_capacity or 4096
        first = max(1, n - cap + 1)
        return self.force_history(which, first, n - first + 1, body)

    def body_state(self, body=1):
        s = BodyState()
        self._chk(self._lib.vplbm_get_body_state_of(self._h, int(body), C.byref(s)))
        return np.array([s.x, s.y, s.theta, s.u, s.v, s.omega])

    def macro_device(self):
        """rho, ux, uy of the last VPLBM_STEP_MACRO step as new device tensors
        [ny][nx] of the compute type, filled on the lattice's stream."""
        import torch

        dt = torch.float64 if self.params.precision == F64 else torch.float32
        out = [torch.empty((self.ny, self.nx), dtype=dt, device="cuda") for _ in range(3)]
        self._chk(self._lib.vplbm_read_macro_device(self._h, *(C.c_void_p(t.data_ptr()) for t in out)))
        return out

    def macro(self):
        r = np.zeros((self.ny, self.nx))
        u = np.zeros((self.ny, self.nx))
        v = np.zeros((self.ny, self.nx))
        self._chk(self._lib.vplbm_read_macro(self._h, _dptr(r), _dptr(u), _dptr(v)))
        return r, u, v

    def macro_window(self, x0, y0, w, h):
        r, u, v = np.zeros((h, w)), np.zeros((h, w)), np.zeros((h, w))
        self._chk(self._lib.vplbm_read_macro_window(self._h, x0, y0, w, h, _dptr(r), _dptr(u), _dptr(v)))
        return r, u, v

    def populations_window(self, x0, y0, w, h):
        """Post-collision populations of a window, float64 (9, h, w)."""
        f = np.zeros((9, h, w))
        self._chk(self._lib.vplbm_read_populations_window(self._h, x0, y0, w, h, _dptr(f)))
        return f

    def populations(self):
        """Post-collision populations as float64, shape (9, ny, nx)."""
        f = np.zeros((9, self.ny, self.nx))
        self._chk(self._lib.vplbm_read_populations(self._h, _dptr(f)))
        return f

    def mask(self):
        m = np.zeros((self.ny, self.nx), np.uint8)
        self._chk(self._lib.vplbm_read_mask(self._h, m.ctypes.data_as(C.POINTER(C.c_uint8))))
        return m


class Batch:
    """Several lattices stepped together, one launch per time step."""

    def __init__(self, lattices):
        self._lib = load_library()
        self.lattices = list(lattices)
        arr = (C.c_void_p * len(self.lattices))(*[l._h.value for l in self.lattices])
        h = C.c_void_p()
        rc = self._lib.vplbm_batch_create(arr, len(self.lattices), C.byref(h))
        if rc != OK:
            raise VplbmError(rc, "vplbm_batch_create failed (same precision, collision, stream and storage "
                                 "scheme required)")
        self._h = h

    def step(self, nsteps):
        n = (C.c_int * len(self.lattices))(*[int(v) for v in nsteps])
        rc = self._lib.vplbm_batch_step(self._h, n)
        if rc != OK:
            raise VplbmError(rc, self._lib.vplbm_batch_last_error(self._h).decode(errors="replace"))

    def set_lattices(self, lattices):
        """Replace the batch's lattices (same precision, collision, stream, storage)."""
        lats = list(lattices)
        arr = (C.c_void_p * len(lats))(*[l._h.value for l in lats])
        rc = self._lib.vplbm_batch_set_lattices(self._h, arr, len(lats))
        if rc != OK:
            raise VplbmError(rc, self._lib.vplbm_batch_last_error(self._h).decode(errors="replace"))
        self.lattices = lats

    def set_tile(self, bx, by):
        rc = self._lib.vplbm_batch_set_tile(self._h, int(bx), int(by))
        if rc != OK:
            raise VplbmError(rc, self._lib.vplbm_batch_last_error(self._h).decode(errors="replace"))

    @property
    def tile(self):
        """(bx, by): the tile of the batched launches."""
        bx, by = C.c_int(0), C.c_int(0)
        rc = self._lib.vplbm_batch_get_tile(self._h, C.byref(bx), C.byref(by))
        if rc != OK:
            raise VplbmError(rc, "vplbm_batch_get_tile failed")
        return bx.value, by.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.vplbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step_noalloc(lattices, nsteps):
    """vplbm_batch_step_noalloc: step the lattices together without any
    device allocation (the library's static tables; see include/vplbm.h)."""
    lib = load_library()
    lats = list(lattices)
    arr = (C.c_void_p * len(lats))(*[l._h.value for l in lats])
    n = (C.c_int * len(lats))(*[int(v) for v in nsteps])
    rc = lib.vplbm_batch_step_noalloc(arr, len(lats), n)
    if rc != OK:
        raise VplbmError(rc, lib.vplbm_last_error(lats[0]._h).decode(errors="replace"))
