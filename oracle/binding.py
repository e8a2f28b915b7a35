"""ctypes binding of the CPU FP64 oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import
this module.  The GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle.cpp")]

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ (FP64, no fast-math, no FMA contraction)."""
    cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c++17", "-fPIC",
           "-shared", "-fopenmp", "-o", LIB_PATH + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Desc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("verts", _dp), ("nt", C.c_int32), ("tets", _ip),
                ("dirichlet", C.POINTER(C.c_uint8)), ("youngs", C.c_double),
                ("poisson", C.c_double), ("density", C.c_double), ("nb", C.c_int32),
                ("body_nv", _ip), ("body_nf", _ip), ("body_verts", _dp), ("body_tris", _ip),
                ("body_density", _dp), ("body_prescribed", _ip), ("h", C.c_double),
                ("dhat", C.c_double), ("kappa", C.c_double), ("kappa_s", C.c_double),
                ("newton_tol", C.c_double), ("gravity", C.c_double * 3),
                ("max_newton", C.c_int32), ("max_al", C.c_int32), ("friction", C.c_double),
                ("eps_v", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("al_rounds", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Desc), C.c_char_p, C.c_int32]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(_Stats)]
        L.orc_step_begin.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_step_finish.argtypes = [C.c_void_p, C.POINTER(_Stats)]
        L.orc_system.argtypes = [C.c_void_p, C.c_uint32, _dp, _dp, C.c_int32, _ip, _ip, _dp,
                                 C.c_int32, _ip, _ip]
        L.orc_newton_direction.argtypes = [C.c_void_p, _dp, C.c_int32]
        L.orc_num_world_verts.argtypes = [C.c_void_p]
        L.orc_scene_scale.argtypes = [C.c_void_p]
        L.orc_scene_scale.restype = C.c_double
        L.orc_diagnostics.argtypes = [C.c_void_p, _dp, _dp, _ip]
        L.orc_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_set_state.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_world_positions.argtypes = [C.c_void_p, _dp]
        L.orc_ls_log.argtypes = [C.c_void_p, _dp, C.c_int32]
        L.orc_newton_log.argtypes = [C.c_void_p, _dp, C.c_int32]
        L.orc_candidates.argtypes = [C.c_void_p, _dp, _dp, _ip, C.c_int32]
        L.orc_nh_tet.argtypes = [_dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp, _dp]
        L.orc_pair_barrier.argtypes = [C.c_int32, _dp, C.c_double, C.c_double, C.c_double,
                                       _dp, _dp, _dp, _dp]
        L.orc_pair_sqdist.argtypes = [C.c_int32, _dp, _ip]
        L.orc_pair_sqdist.restype = C.c_double
        L.orc_accd.argtypes = [C.c_int32, _dp, _dp, C.c_double, C.c_int32]
        L.orc_accd.restype = C.c_double
        L.orc_barrier.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.orc_barrier.restype = C.c_double
        L.orc_abd_mass.argtypes = [C.c_int32, _dp, C.c_int32, _ip, C.c_double, _dp]
        L.orc_arap.argtypes = [_dp, _dp, _dp, _dp]
        L.orc_arap.restype = C.c_double
        L.orc_psd_project.argtypes = [C.c_int32, _dp, _dp]
        L.orc_pair_friction.argtypes = [C.c_int32, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_double, _dp, _dp, _dp]
        L.orc_pair_friction.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleScene:
    """One scene of the oracle, built from a ``scenes.SceneSpec``."""

    STATUS = {0: "OK", 3: "NOT_CONVERGED", 4: "LINESEARCH_FAILED", 5: "AL_FAILED", 6: "NAN",
              7: "INFEASIBLE_TARGET"}

    def __init__(self, spec, max_newton=None, max_al=None):
        self.spec = spec
        self._keep = []
        verts = _f64(spec.verts)
        tets = np.ascontiguousarray(spec.tets, dtype=np.int32)
        dirich = np.ascontiguousarray(spec.dirichlet, dtype=np.uint8)
        nb = len(spec.bodies)
        bnv = np.array([len(b.verts) for b in spec.bodies] or [0], dtype=np.int32)
        bnf = np.array([len(b.tris) for b in spec.bodies] or [0], dtype=np.int32)
        bv = _f64(np.concatenate([b.verts for b in spec.bodies]) if nb else np.zeros((1, 3)))
        bt = np.ascontiguousarray(np.concatenate([b.tris for b in spec.bodies]) if nb
                                  else np.zeros((1, 3)), dtype=np.int32)
        bd = np.array([b.density for b in spec.bodies] or [0.0], dtype=np.float64)
        bp = np.array([1 if b.prescribed else 0 for b in spec.bodies] or [0], dtype=np.int32)
        self._keep += [verts, tets, dirich, bnv, bnf, bv, bt, bd, bp]
        p = spec.params
        d = _Desc()
        d.nv = len(verts)
        d.verts = _d(verts)
        d.nt = len(tets)
        d.tets = _i(tets)
        d.dirichlet = dirich.ctypes.data_as(C.POINTER(C.c_uint8))
        d.youngs, d.poisson, d.density = spec.youngs, spec.poisson, spec.density
        d.nb = nb
        d.body_nv, d.body_nf, d.body_verts, d.body_tris = _i(bnv), _i(bnf), _d(bv), _i(bt)
        d.body_density, d.body_prescribed = _d(bd), _i(bp)
        d.h, d.dhat, d.kappa, d.kappa_s = p["h"], p["dhat"], p["kappa"], p["kappa_s"]
        d.newton_tol = p["newton_tol"]
        d.gravity = (C.c_double * 3)(*p["gravity"])
        d.max_newton = max_newton or p.get("max_newton", 100)
        d.max_al = max_al or p.get("max_al", 30)
        d.friction = p.get("friction", 0.0)
        d.eps_v = p.get("eps_v", 0.0)
        err = C.create_string_buffer(256)
        self.h = lib().orc_create(C.byref(d), err, 256)
        if not self.h:
            raise ValueError("oracle create failed: " + err.value.decode())
        self.nv = d.nv
        self.nb = nb
        self.nw = lib().orc_num_world_verts(self.h)
        self.scale = lib().orc_scene_scale(self.h)
        self.n_moving = int((dirich == 2).sum())

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def step(self, k=None, body_targets=None, dir_targets=None):
        if body_targets is None:
            body_targets = self.spec.body_targets[k]
        if dir_targets is None:
            dir_targets = (self.spec.dirichlet_targets[k] if self.n_moving
                           else np.zeros((1, 3)))
        bt = _f64(np.asarray(body_targets).reshape(-1) if self.nb else np.zeros(12))
        dt = _f64(np.asarray(dir_targets).reshape(-1) if self.n_moving else np.zeros(3))
        st = _Stats()
        rc = lib().orc_step(self.h, _d(bt), _d(dt), C.byref(st))
        return rc, dict(status=st.status, newton_iters=st.newton_iters,
                        al_rounds=st.al_rounds)

    def _targets(self, k, body_targets, dir_targets):
        if body_targets is None:
            body_targets = self.spec.body_targets[k]
        if dir_targets is None:
            dir_targets = (self.spec.dirichlet_targets[k] if self.n_moving
                           else np.zeros((1, 3)))
        bt = _f64(np.asarray(body_targets).reshape(-1) if self.nb else np.zeros(12))
        dt = _f64(np.asarray(dir_targets).reshape(-1) if self.n_moving else np.zeros(3))
        return bt, dt

    def step_begin(self, k=None, body_targets=None, dir_targets=None):
        bt, dt = self._targets(k, body_targets, dir_targets)
        return lib().orc_step_begin(self.h, _d(bt), _d(dt))

    def step_finish(self):
        st = _Stats()
        rc = lib().orc_step_finish(self.h, C.byref(st))
        return rc, dict(status=st.status, newton_iters=st.newton_iters,
                        al_rounds=st.al_rounds)

    TERMS = dict(inertia=1, elastic=2, body_stiffness=4, constraint=8, contact=16, friction=32,
                 all=63)

    def system(self, terms="all"):
        """Newton system of the current state: (energy, G[n_nodes, 3], blocks dict
        {(row, col): 3x3}, node_of[nv + nb])."""
        t = self.TERMS[terms] if isinstance(terms, str) else int(terms)
        e = C.c_double()
        nblk = C.c_int32()
        node_of = np.zeros(self.nv + max(self.nb, 1), dtype=np.int32)
        nn = lib().orc_system(self.h, t, C.byref(e), None, 0, None, None, None, 0,
                              C.byref(nblk), None)
        G = np.zeros(max(3 * nn, 1))
        nb = nblk.value
        rows = np.zeros(max(nb, 1), dtype=np.int32)
        cols = np.zeros(max(nb, 1), dtype=np.int32)
        vals = np.zeros((max(nb, 1), 9))
        lib().orc_system(self.h, t, C.byref(e), _d(G), 3 * nn, _i(rows), _i(cols), _d(vals), nb,
                         C.byref(nblk), _i(node_of))
        blocks = {(int(r), int(c)): vals[k].reshape(3, 3) for k, (r, c) in
                  enumerate(zip(rows[:nb], cols[:nb]))}
        return e.value, G[:3 * nn].reshape(-1, 3), blocks, node_of[:self.nv + self.nb]

    def newton_direction(self):
        nn = lib().orc_newton_direction(self.h, None, 0)
        if nn < 0:
            raise RuntimeError("oracle factorisation broke down")
        p = np.zeros(max(3 * nn, 1))
        lib().orc_newton_direction(self.h, _d(p), 3 * nn)
        return p[:3 * nn].reshape(-1, 3)

    def get_state(self):
        x = np.zeros((self.nv, 3))
        v = np.zeros((self.nv, 3))
        q = np.zeros((max(self.nb, 1), 12))
        qd = np.zeros((max(self.nb, 1), 12))
        lib().orc_get_state(self.h, _d(x), _d(v), _d(q), _d(qd))
        return x, v, q[:self.nb], qd[:self.nb]

    def set_state(self, x, v, q, qd):
        x, v = _f64(x), _f64(v)
        q = _f64(q if self.nb else np.zeros((1, 12)))
        qd = _f64(qd if self.nb else np.zeros((1, 12)))
        lib().orc_set_state(self.h, _d(x), _d(v), _d(q), _d(qd))

    def world_positions(self):
        out = np.zeros((self.nw, 3))
        lib().orc_world_positions(self.h, _d(out))
        return out

    def diagnostics(self):
        dmin = C.c_double()
        jmin = C.c_double()
        nact = C.c_int32()
        lib().orc_diagnostics(self.h, C.byref(dmin), C.byref(jmin), C.byref(nact))
        return dmin.value, jmin.value, nact.value

    def ls_log(self):
        n = lib().orc_ls_log(self.h, None, 0)
        out = np.zeros(max(n, 1))
        lib().orc_ls_log(self.h, _d(out), n)
        return out[:n].reshape(-1, 2)

    def newton_log(self):
        """Per Newton iteration of the last step: (AL round, iteration, max |p|, CCD bound,
        step size, active pairs, max kappa_A, max body residual)."""
        n = lib().orc_newton_log(self.h, None, 0)
        out = np.zeros(max(n, 1))
        lib().orc_newton_log(self.h, _d(out), n)
        return out[:n].reshape(-1, 8)

    def candidates(self, P0, P1=None):
        P0 = _f64(P0)
        P1c = _f64(P1) if P1 is not None else None
        n = lib().orc_candidates(self.h, _d(P0), _d(P1c) if P1c is not None else None,
                                 None, 0)
        out = np.zeros((max(n, 1), 5), dtype=np.int32)
        lib().orc_candidates(self.h, _d(P0), _d(P1c) if P1c is not None else None,
                             _i(out), n)
        return out[:n]


# ------------------------------------------------------------------ pure evaluators
def nh_tet(rest, x, mu, lam):
    rest, x = _f64(rest).reshape(12), _f64(x).reshape(12)
    e = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros(144)
    Hp = np.zeros(144)
    lib().orc_nh_tet(_d(rest), _d(x), mu, lam, _d(e), _d(g), _d(H), _d(Hp))
    return e[0], g, H.reshape(12, 12), Hp.reshape(12, 12)


def pair_barrier(kind, x, meps, dhat, kappa):
    x = _f64(x).reshape(12)
    e = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros(144)
    Hp = np.zeros(144)
    t = lib().orc_pair_barrier(kind, _d(x), meps, dhat, kappa, _d(e), _d(g), _d(H), _d(Hp))
    return e[0], g, H.reshape(12, 12), Hp.reshape(12, 12), t


def pair_friction(kind, xn, x, meps, dhat, kappa, mu, eps_v_h):
    """Friction potential of one pair lagged at xn, at x: (lambda, e, g, H)."""
    xn = _f64(xn).reshape(12)
    x = _f64(x).reshape(12)
    e = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros(144)
    lam = lib().orc_pair_friction(kind, _d(xn), _d(x), meps, dhat, kappa, mu, eps_v_h, _d(e),
                                  _d(g), _d(H))
    return lam, e[0], g, H.reshape(12, 12)


def pair_sqdist(kind, x):
    x = _f64(x).reshape(12)
    t = C.c_int32()
    s = lib().orc_pair_sqdist(kind, _d(x), C.byref(t))
    return s, t.value


def accd(kind, x, p, gap_ratio=0.1, max_iter=100000):
    x, p = _f64(x).reshape(12), _f64(p).reshape(12)
    return lib().orc_accd(kind, _d(x), _d(p), gap_ratio, max_iter)


def barrier(d, dhat):
    d1 = C.c_double()
    d2 = C.c_double()
    b = lib().orc_barrier(d, dhat, C.byref(d1), C.byref(d2))
    return b, d1.value, d2.value


def abd_mass(verts, tris, rho):
    v = _f64(verts)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    out = np.zeros(14)
    lib().orc_abd_mass(len(v), _d(v), len(t), _i(t), rho, _d(out))
    return dict(m=out[0], volume=out[1], com=out[2:5], Q=out[5:14].reshape(3, 3))


def arap(A):
    A = _f64(A).reshape(9)
    g = np.zeros(9)
    H = np.zeros(81)
    Hp = np.zeros(81)
    e = lib().orc_arap(_d(A), _d(g), _d(H), _d(Hp))
    return e, g.reshape(3, 3), H.reshape(9, 9), Hp.reshape(9, 9)


def psd_project(A):
    A = _f64(A)
    n = A.shape[0]
    out = np.zeros_like(A)
    lib().orc_psd_project(n, _d(A), _d(out))
    return out
