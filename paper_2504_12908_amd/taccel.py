"""Thin ctypes binding of libtaccel (argument marshalling only).

Names follow include/taccel.h.  Every step of a time step runs in the library's HIP
kernels; this module only converts numpy arrays and ``scenes.SceneSpec`` objects to the C
structures.  It refuses to work without the built library (no CPU fallback exists).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtaccel.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)

OK, ERR_ARG, ERR_HIP, NOT_CONVERGED, LINESEARCH_FAILED, AL_FAILED, NAN, INFEASIBLE_TARGET, \
    ERR_OOM, INFEASIBLE, CANCELLED = range(11)
FP64, MIXED, FP64_REFINED = 0, 1, 2
FIELD_X, FIELD_V, FIELD_Q, FIELD_QDOT, FIELD_BODY_X, FIELD_CONTACTS, FIELD_STATS = range(7)
STATUS_NAMES = ["OK", "ERR_ARG", "ERR_HIP", "NOT_CONVERGED", "LINESEARCH_FAILED", "AL_FAILED",
                "NAN", "INFEASIBLE_TARGET", "ERR_OOM", "INFEASIBLE", "CANCELLED"]


class taccel_soft_desc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("verts", _dp), ("nt", C.c_int32), ("tets", _ip),
                ("dirichlet", C.POINTER(C.c_uint8)), ("youngs", C.c_double),
                ("poisson", C.c_double), ("density", C.c_double)]


class taccel_body_desc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("verts", _dp), ("nf", C.c_int32), ("tris", _ip),
                ("density", C.c_double), ("prescribed", C.c_int32)]


class taccel_camera(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("axis_u", C.c_double * 3),
                ("axis_v", C.c_double * 3), ("pixel", C.c_double), ("width", C.c_int32),
                ("height", C.c_int32)]


def camera(origin, axis_u, axis_v, pixel, width, height):
    """An image plane for depth maps (see taccel_camera)."""
    c = taccel_camera()
    c.origin = (C.c_double * 3)(*origin)
    c.axis_u = (C.c_double * 3)(*axis_u)
    c.axis_v = (C.c_double * 3)(*axis_v)
    c.pixel = pixel
    c.width, c.height = int(width), int(height)
    return c


def _markers(fn, args, tris, bary):
    tris = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    bary = _f64(bary).reshape(-1, 3)
    m = len(tris)
    pos, flow = np.zeros((m, 3)), np.zeros((m, 3))
    _check(fn(*args, m, _i(tris), _d(bary), _d(pos), _d(flow)), "markers")
    return pos, flow


def _depth_map(fn, args, cam, tris):
    tris = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    depth = np.zeros((cam.height, cam.width))
    normal = np.zeros((cam.height, cam.width, 3))
    _check(fn(*args, C.byref(cam), len(tris), _i(tris), _d(depth), _d(normal)), "depth_map")
    return depth, normal


class taccel_params(C.Structure):
    _fields_ = [("h", C.c_double), ("dhat", C.c_double), ("kappa", C.c_double),
                ("kappa_s", C.c_double), ("newton_tol", C.c_double),
                ("gravity", C.c_double * 3), ("max_newton", C.c_int32), ("max_al", C.c_int32),
                ("max_pcg", C.c_int32), ("pcg_eta", C.c_double), ("precision", C.c_int32),
                ("friction", C.c_double), ("eps_v", C.c_double), ("pcg_forcing", C.c_int32)]


class taccel_scene_desc(C.Structure):
    _fields_ = [("soft", taccel_soft_desc), ("n_bodies", C.c_int32),
                ("bodies", C.POINTER(taccel_body_desc)), ("params", taccel_params)]


_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class taccel_runtime(C.Structure):
    _fields_ = [("alloc", _ALLOC), ("free", _FREE), ("ctx", C.c_void_p), ("stream", C.c_void_p)]


class taccel_targets(C.Structure):
    _fields_ = [("body_targets", _dp), ("dirichlet_targets", _dp)]


class taccel_step_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("al_rounds", C.c_int32),
                ("pcg_iters", C.c_int32), ("n_active", C.c_int32), ("ls_halvings", C.c_int32),
                ("step_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class taccel_server_params(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_double), ("max_cohort", C.c_int32),
                ("max_cohorts", C.c_int32), ("coalesce_ms", C.c_double)]


class taccel_completion(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("status", C.c_int32), ("n_steps", C.c_int32),
                ("steps_done", C.c_int32), ("wait_ms", C.c_double), ("run_ms", C.c_double),
                ("mean_step_ms", C.c_double), ("max_step_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libtaccel.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2504_12908_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        L.taccel_last_error.restype = C.c_char_p
        L.taccel_status_str.restype = C.c_char_p
        L.taccel_scene_create.argtypes = [C.POINTER(taccel_scene_desc), C.POINTER(taccel_runtime),
                                          C.POINTER(C.c_void_p)]
        L.taccel_step.argtypes = [C.c_void_p, C.POINTER(taccel_targets),
                                  C.POINTER(taccel_step_stats)]
        L.taccel_state_read.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]
        L.taccel_state_write.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]
        L.taccel_scene_destroy.argtypes = [C.c_void_p]
        L.taccel_batch_create.argtypes = [C.POINTER(taccel_scene_desc), C.c_int32,
                                          C.POINTER(taccel_runtime), C.POINTER(C.c_void_p)]
        L.taccel_batch_step.argtypes = [C.c_void_p, C.POINTER(taccel_targets), _ip,
                                        C.POINTER(taccel_step_stats)]
        L.taccel_batch_read.argtypes = [C.c_void_p, C.c_int32, C.c_int, C.c_void_p, C.c_size_t]
        L.taccel_batch_write.argtypes = [C.c_void_p, C.c_int32, C.c_int, C.c_void_p, C.c_size_t]
        L.taccel_batch_destroy.argtypes = [C.c_void_p]
        L.taccel_state_bytes.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_size_t)]
        L.taccel_batch_state_bytes.argtypes = [C.c_void_p, C.c_int32, C.c_int, C.POINTER(C.c_size_t)]
        L.taccel_state_read_device.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]
        L.taccel_batch_read_device.argtypes = [C.c_void_p, C.c_int32, C.c_int, C.c_void_p,
                                               C.c_size_t]
        L.taccel_scene_reset.argtypes = [C.c_void_p]
        L.taccel_batch_reset.argtypes = [C.c_void_p, C.POINTER(C.c_uint8)]
        L.taccel_debug_fem.argtypes = [C.c_int32, _dp, _dp, C.c_double, C.c_double, _dp, _dp,
                                       _dp, _dp]
        L.taccel_debug_barrier.argtypes = [C.c_int32, _ip, _dp, _dp, C.c_double, C.c_double,
                                           _dp, _dp, _dp, _dp, _ip]
        L.taccel_debug_ccd.argtypes = [C.c_int32, _ip, _dp, _dp, C.c_double, C.c_int32, _dp]
        L.taccel_markers.argtypes = [C.c_void_p, C.c_int32, _ip, _dp, _dp, _dp]
        L.taccel_batch_markers.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _ip, _dp, _dp, _dp]
        L.taccel_depth_map.argtypes = [C.c_void_p, C.POINTER(taccel_camera), C.c_int32, _ip,
                                       _dp, _dp]
        L.taccel_batch_depth_map.argtypes = [C.c_void_p, C.c_int32, C.POINTER(taccel_camera),
                                             C.c_int32, _ip, _dp, _dp]
        L.taccel_debug_friction.argtypes = [C.c_int32, _ip, _dp, _dp, _dp, C.c_double,
                                            C.c_double, C.c_double, C.c_double, _dp, _dp, _dp,
                                            _dp]
        L.taccel_debug_arap.argtypes = [C.c_int32, _dp, _dp, _dp, _dp, _dp]
        L.taccel_debug_candidates.argtypes = [C.c_void_p, _dp, _dp, _ip, C.c_int32, _ip]
        L.taccel_debug_system.argtypes = [C.c_void_p, C.POINTER(taccel_targets), _dp, _ip, _ip,
                                          _dp, C.c_int32, _ip]
        L.taccel_server_create.argtypes = [C.POINTER(taccel_server_params),
                                           C.POINTER(taccel_runtime), C.POINTER(C.c_void_p)]
        L.taccel_server_submit.argtypes = [C.c_void_p, C.POINTER(taccel_scene_desc), C.c_int32,
                                           C.POINTER(taccel_targets), C.POINTER(C.c_uint64)]
        L.taccel_server_poll.argtypes = [C.c_void_p, C.POINTER(taccel_completion), C.c_int32,
                                         _ip, C.c_int32]
        L.taccel_server_read.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.c_void_p, C.c_size_t]
        L.taccel_server_step_latencies.argtypes = [C.c_void_p, C.c_uint64, _dp, C.c_int32, _ip]
        L.taccel_server_release.argtypes = [C.c_void_p, C.c_uint64]
        L.taccel_server_info.argtypes = [C.c_void_p, _ip, _ip, _dp, _dp]
        L.taccel_server_destroy.argtypes = [C.c_void_p]
        L.taccel_profile_enable.argtypes = [C.c_int32]
        L.taccel_profile_query.argtypes = [C.c_char_p, _dp, C.POINTER(C.c_int64), _dp]
        _lib = L
    return _lib


class TaccelError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().taccel_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")


def _check(status, where):
    if status != OK:
        raise TaccelError(status, where)


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _Desc:
    """C description of one SceneSpec (keeps the numpy buffers alive)."""

    def __init__(self, spec, precision=FP64, overrides=None):
        p = dict(spec.params)
        p.update(overrides or {})
        self.keep = []
        verts = _f64(spec.verts)
        tets = np.ascontiguousarray(spec.tets, dtype=np.int32)
        dirich = np.ascontiguousarray(spec.dirichlet, dtype=np.uint8)
        self.keep += [verts, tets, dirich]
        d = taccel_scene_desc()
        d.soft.nv = len(verts)
        d.soft.verts = _d(verts)
        d.soft.nt = len(tets)
        d.soft.tets = _i(tets)
        d.soft.dirichlet = dirich.ctypes.data_as(C.POINTER(C.c_uint8))
        d.soft.youngs, d.soft.poisson, d.soft.density = spec.youngs, spec.poisson, spec.density
        nb = len(spec.bodies)
        bodies = (taccel_body_desc * max(nb, 1))()
        for k, b in enumerate(spec.bodies):
            bv = _f64(b.verts)
            bt = np.ascontiguousarray(b.tris, dtype=np.int32)
            self.keep += [bv, bt]
            bodies[k].nv = len(bv)
            bodies[k].verts = _d(bv)
            bodies[k].nf = len(bt)
            bodies[k].tris = _i(bt)
            bodies[k].density = b.density
            bodies[k].prescribed = 1 if b.prescribed else 0
        self.keep.append(bodies)
        d.n_bodies = nb
        d.bodies = C.cast(bodies, C.POINTER(taccel_body_desc))
        d.params.h, d.params.dhat, d.params.kappa = p["h"], p["dhat"], p["kappa"]
        d.params.kappa_s, d.params.newton_tol = p["kappa_s"], p["newton_tol"]
        d.params.gravity = (C.c_double * 3)(*p["gravity"])
        d.params.max_newton = p.get("max_newton", 100)
        d.params.max_al = p.get("max_al", 30)
        d.params.max_pcg = p.get("max_pcg", 10000)
        d.params.pcg_eta = overrides.get("pcg_eta", 0.0) if overrides else 0.0
        d.params.precision = precision
        d.params.friction = p.get("friction", 0.0)
        d.params.eps_v = p.get("eps_v", 0.0)
        d.params.pcg_forcing = int(p.get("pcg_forcing", 0))
        self.desc = d
        self.nv = len(verts)
        self.nb = nb
        self.n_moving = int((dirich == 2).sum())
        self.body_nv = [len(b.verts) for b in spec.bodies]


class _Targets:
    def __init__(self, spec, k, body_targets=None, dirichlet_targets=None):
        if body_targets is None and len(spec.bodies):
            body_targets = spec.body_targets[k]
        if dirichlet_targets is None and int((spec.dirichlet == 2).sum()):
            dirichlet_targets = spec.dirichlet_targets[k]
        self.bt = _f64(body_targets).reshape(-1) if body_targets is not None else None
        self.dt = _f64(dirichlet_targets).reshape(-1) if dirichlet_targets is not None else None
        self.t = taccel_targets()
        self.t.body_targets = _d(self.bt) if self.bt is not None and self.bt.size else None
        self.t.dirichlet_targets = _d(self.dt) if self.dt is not None and self.dt.size else None


def _runtime(stream):
    if stream is None:
        return None
    rt = taccel_runtime()
    rt.stream = stream
    return rt


def _field_shape(desc, field):
    if field in (FIELD_X, FIELD_V):
        return (desc.nv, 3)
    if field in (FIELD_Q, FIELD_QDOT):
        return (desc.nb, 12)
    return (sum(desc.body_nv), 3)


def _read_contacts(bytes_fn, read_fn, head):
    nb = C.c_size_t()
    _check(bytes_fn(*head, FIELD_CONTACTS, C.byref(nb)), "state_bytes")
    out = np.zeros((nb.value // 20, 5), dtype=np.int32)
    _check(read_fn(*head, FIELD_CONTACTS, out.ctypes.data if out.size else None, nb.value),
           "state_read")
    return out


class Scene:
    """One scene on the GPU (taccel_scene_*)."""

    def __init__(self, spec, precision=FP64, stream=None, **overrides):
        self.spec = spec
        self._d = _Desc(spec, precision, overrides)
        self._rt = _runtime(stream)
        h = C.c_void_p()
        _check(lib().taccel_scene_create(C.byref(self._d.desc),
                                         C.byref(self._rt) if self._rt else None, C.byref(h)),
               "taccel_scene_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().taccel_scene_destroy(self.h)
            self.h = None

    __del__ = close

    def step(self, k=None, body_targets=None, dirichlet_targets=None):
        t = _Targets(self.spec, k, body_targets, dirichlet_targets)
        st = taccel_step_stats()
        rc = lib().taccel_step(self.h, C.byref(t.t), C.byref(st))
        return rc, st.as_dict()

    def read(self, field):
        out = np.zeros(_field_shape(self._d, field))
        _check(lib().taccel_state_read(self.h, field, out.ctypes.data, out.nbytes), "state_read")
        return out

    def write(self, field, arr):
        a = _f64(arr)
        _check(lib().taccel_state_write(self.h, field, a.ctypes.data, a.nbytes), "state_write")

    def get_state(self):
        return (self.read(FIELD_X), self.read(FIELD_V), self.read(FIELD_Q),
                self.read(FIELD_QDOT))

    def contacts(self):
        """Pairs closer than dhat at the current positions: (n, 5) int32 records."""
        return _read_contacts(lib().taccel_state_bytes, lib().taccel_state_read, (self.h,))

    def stats(self):
        """taccel_step_stats of the last step (FIELD_STATS)."""
        st = taccel_step_stats()
        _check(lib().taccel_state_read(self.h, FIELD_STATS, C.addressof(st), C.sizeof(st)),
               "state_read")
        return st.as_dict()

    def read_device(self, field, ptr, nbytes):
        """Write a field to device memory at address ptr (taccel_state_read_device)."""
        _check(lib().taccel_state_read_device(self.h, field, C.c_void_p(ptr), nbytes),
               "state_read_device")

    def field_shape(self, field):
        return _field_shape(self._d, field)

    def reset(self):
        _check(lib().taccel_scene_reset(self.h), "scene_reset")

    def set_state(self, x, v, q, qd):
        self.write(FIELD_X, x)
        self.write(FIELD_V, v)
        if self._d.nb:
            self.write(FIELD_Q, q)
            self.write(FIELD_QDOT, qd)

    def markers(self, tris, bary):
        """Marker positions and flows (m, 3) each (taccel_markers)."""
        return _markers(lib().taccel_markers, (self.h,), tris, bary)

    def depth_map(self, cam, tris):
        """Depth (H, W) and normal (H, W, 3) maps of the surface ``tris`` (taccel_depth_map)."""
        return _depth_map(lib().taccel_depth_map, (self.h,), cam, tris)

    def debug_system(self, k=None, body_targets=None, dirichlet_targets=None):
        """Newton system of the first iteration of step k (taccel_debug_system): gradient
        (nv + 4 nb, 3) and {(row, col): 3x3} blocks in the caller's node numbering."""
        t = _Targets(self.spec, k, body_targets, dirichlet_targets)
        nn = self._d.nv + 4 * self._d.nb
        grad = np.zeros((nn, 3))
        n = C.c_int32()
        _check(lib().taccel_debug_system(self.h, C.byref(t.t), _d(grad), None, None, None, 0,
                                         C.byref(n)), "debug_system")
        cap = n.value
        rows = np.zeros(max(cap, 1), dtype=np.int32)
        cols = np.zeros(max(cap, 1), dtype=np.int32)
        vals = np.zeros((max(cap, 1), 9))
        _check(lib().taccel_debug_system(self.h, C.byref(t.t), _d(grad), _i(rows), _i(cols),
                                         _d(vals), cap, C.byref(n)), "debug_system")
        blocks = {(int(r), int(c)): vals[i].reshape(3, 3)
                  for i, (r, c) in enumerate(zip(rows[:n.value], cols[:n.value]))}
        return grad, blocks

    def candidates(self, P0, P1=None):
        P0 = _f64(P0)
        P1c = _f64(P1) if P1 is not None else None
        n = C.c_int32()
        _check(lib().taccel_debug_candidates(self.h, _d(P0), _d(P1c) if P1c is not None else None,
                                             None, 0, C.byref(n)), "debug_candidates")
        out = np.zeros((max(n.value, 1), 5), dtype=np.int32)
        _check(lib().taccel_debug_candidates(self.h, _d(P0), _d(P1c) if P1c is not None else None,
                                             _i(out), n.value, C.byref(n)), "debug_candidates")
        return out[:n.value]


class Batch:
    """Several independent scenes solved together (taccel_batch_*)."""

    def __init__(self, specs, precision=FP64, stream=None, **overrides):
        self.specs = list(specs)
        self._ds = [_Desc(s, precision, overrides) for s in self.specs]
        arr = (taccel_scene_desc * len(self._ds))(*[d.desc for d in self._ds])
        self._arr = arr
        self._rt = _runtime(stream)
        h = C.c_void_p()
        _check(lib().taccel_batch_create(arr, len(self._ds),
                                         C.byref(self._rt) if self._rt else None, C.byref(h)),
               "taccel_batch_create")
        self.h = h
        self.n = len(self._ds)

    def close(self):
        if getattr(self, "h", None):
            lib().taccel_batch_destroy(self.h)
            self.h = None

    __del__ = close

    def targets(self, k):
        """Targets of step k of every scene's script, marshalled once (pass to step)."""
        ts = [_Targets(s, k) for s in self.specs]
        return ts, (taccel_targets * self.n)(*[t.t for t in ts])

    def step(self, k, targets=None):
        ts, arr = targets if targets is not None else self.targets(k)
        per = np.zeros(self.n, dtype=np.int32)
        st = (taccel_step_stats * self.n)()
        rc = lib().taccel_batch_step(self.h, arr, _i(per), st)
        return rc, per, [s.as_dict() for s in st]

    def read(self, i, field):
        out = np.zeros(_field_shape(self._ds[i], field))
        _check(lib().taccel_batch_read(self.h, i, field, out.ctypes.data, out.nbytes),
               "batch_read")
        return out

    def write(self, i, field, arr):
        a = _f64(arr)
        _check(lib().taccel_batch_write(self.h, i, field, a.ctypes.data, a.nbytes), "batch_write")

    def contacts(self, i):
        return _read_contacts(lib().taccel_batch_state_bytes, lib().taccel_batch_read, (self.h, i))

    def stats(self, i):
        st = taccel_step_stats()
        _check(lib().taccel_batch_read(self.h, i, FIELD_STATS, C.addressof(st), C.sizeof(st)),
               "batch_read")
        return st.as_dict()

    def read_device(self, i, field, ptr, nbytes):
        _check(lib().taccel_batch_read_device(self.h, i, field, C.c_void_p(ptr), nbytes),
               "batch_read_device")

    def reset(self, mask=None):
        """Creation state for the scenes with mask[k] true (all when mask is None)."""
        m = None
        if mask is not None:
            mm = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
            assert mm.shape == (self.n,)
            m = mm.ctypes.data_as(C.POINTER(C.c_uint8))
        _check(lib().taccel_batch_reset(self.h, m), "batch_reset")

    def markers(self, i, tris, bary):
        return _markers(lib().taccel_batch_markers, (self.h, i), tris, bary)

    def depth_map(self, i, cam, tris):
        return _depth_map(lib().taccel_batch_depth_map, (self.h, i), cam, tris)


class Server:
    """Continuous-batching server of rollout requests (taccel_server_*)."""

    def __init__(self, hbm_budget_bytes, max_cohort=64, max_cohorts=8, coalesce_ms=1.0):
        p = taccel_server_params(float(hbm_budget_bytes), int(max_cohort), int(max_cohorts),
                                 float(coalesce_ms))
        h = C.c_void_p()
        _check(lib().taccel_server_create(C.byref(p), None, C.byref(h)), "taccel_server_create")
        self.h = h
        self._desc = {}

    def close(self):
        if getattr(self, "h", None):
            lib().taccel_server_destroy(self.h)
            self.h = None

    __del__ = close

    def submit(self, spec, n_steps=None, first_step=0, precision=FP64, **overrides):
        """Queue steps first_step .. first_step + n_steps - 1 of spec's target script."""
        n_steps = spec.n_steps - first_step if n_steps is None else n_steps
        d = _Desc(spec, precision, overrides)
        ts = [_Targets(spec, first_step + k) for k in range(n_steps)]
        arr = (taccel_targets * n_steps)(*[t.t for t in ts])
        rid = C.c_uint64()
        _check(lib().taccel_server_submit(self.h, C.byref(d.desc), n_steps, arr, C.byref(rid)),
               "taccel_server_submit")
        self._desc[rid.value] = d
        return rid.value

    def poll(self, cap=64, wait_ms=0):
        out = (taccel_completion * cap)()
        n = C.c_int32()
        _check(lib().taccel_server_poll(self.h, out, cap, C.byref(n), int(wait_ms)), "server_poll")
        return [out[i].as_dict() for i in range(n.value)]

    def read(self, rid, field):
        out = np.zeros(_field_shape(self._desc[rid], field))
        _check(lib().taccel_server_read(self.h, rid, field, out.ctypes.data, out.nbytes),
               "server_read")
        return out

    def step_latencies(self, rid):
        n = C.c_int32()
        _check(lib().taccel_server_step_latencies(self.h, rid, None, 0, C.byref(n)),
               "server_step_latencies")
        out = np.zeros(max(n.value, 1))
        _check(lib().taccel_server_step_latencies(self.h, rid, _d(out), n.value, C.byref(n)),
               "server_step_latencies")
        return out[:n.value]

    def release(self, rid):
        _check(lib().taccel_server_release(self.h, rid), "server_release")
        self._desc.pop(rid, None)

    def info(self):
        q, c = C.c_int32(), C.c_int32()
        u, pk = C.c_double(), C.c_double()
        _check(lib().taccel_server_info(self.h, C.byref(q), C.byref(c), C.byref(u), C.byref(pk)),
               "server_info")
        return dict(queued=q.value, running_cohorts=c.value, used_bytes=u.value,
                    peak_bytes=pk.value)


# ------------------------------------------------------------------ measurement
PHASES = ("candidates", "derivatives", "solve", "check", "ccd", "line_search")


def profile_enable(on=True, phases=False):
    """Kernel timing (spmv, pcg) when on; host wall time per Newton phase when phases."""
    lib().taccel_profile_enable((1 if on else 0) | (2 if phases else 0))


def profile_reset():
    lib().taccel_profile_reset()


def profile_query(kernel="spmv"):
    ms = C.c_double()
    n = C.c_int64()
    b = C.c_double()
    _check(lib().taccel_profile_query(kernel.encode(), C.byref(ms), C.byref(n), C.byref(b)),
           "profile_query")
    return dict(total_ms=ms.value, launches=n.value, bytes=b.value)


def device_synchronize():
    _check(lib().taccel_device_synchronize(), "device_synchronize")


# ------------------------------------------------------------------ element evaluators
def debug_fem(rest, x, youngs, poisson):
    rest, x = _f64(rest).reshape(-1, 12), _f64(x).reshape(-1, 12)
    n = len(rest)
    e, g, H, Hp = np.zeros(n), np.zeros((n, 12)), np.zeros((n, 12, 12)), np.zeros((n, 12, 12))
    _check(lib().taccel_debug_fem(n, _d(rest), _d(x), youngs, poisson, _d(e), _d(g), _d(H),
                                  _d(Hp)), "debug_fem")
    return e, g, H, Hp


def debug_barrier(kinds, x, meps, dhat, kappa):
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    x, meps = _f64(x).reshape(-1, 12), _f64(meps)
    n = len(kinds)
    e, g, H, Hp = np.zeros(n), np.zeros((n, 12)), np.zeros((n, 12, 12)), np.zeros((n, 12, 12))
    t = np.zeros(n, dtype=np.int32)
    _check(lib().taccel_debug_barrier(n, _i(kinds), _d(x), _d(meps), dhat, kappa, _d(e), _d(g),
                                      _d(H), _d(Hp), _i(t)), "debug_barrier")
    return e, g, H, Hp, t


def debug_friction(kinds, xn, x, meps, dhat, kappa, mu, eps_v_h):
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    xn, x, meps = _f64(xn).reshape(-1, 12), _f64(x).reshape(-1, 12), _f64(meps)
    n = len(kinds)
    lam, e, g, H = np.zeros(n), np.zeros(n), np.zeros((n, 12)), np.zeros((n, 12, 12))
    _check(lib().taccel_debug_friction(n, _i(kinds), _d(xn), _d(x), _d(meps), dhat, kappa, mu,
                                       eps_v_h, _d(lam), _d(e), _d(g), _d(H)), "debug_friction")
    return lam, e, g, H


def debug_ccd(kinds, x, p, gap_ratio=0.1, max_iter=100000):
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    x, p = _f64(x).reshape(-1, 12), _f64(p).reshape(-1, 12)
    t = np.zeros(len(kinds))
    _check(lib().taccel_debug_ccd(len(kinds), _i(kinds), _d(x), _d(p), gap_ratio, max_iter,
                                  _d(t)), "debug_ccd")
    return t


def debug_arap(A):
    A = _f64(A).reshape(-1, 9)
    n = len(A)
    e, g, H, Hp = np.zeros(n), np.zeros((n, 9)), np.zeros((n, 9, 9)), np.zeros((n, 9, 9))
    _check(lib().taccel_debug_arap(n, _d(A), _d(e), _d(g), _d(H), _d(Hp)), "debug_arap")
    return e, g.reshape(n, 3, 3), H, Hp
