"""Seeded synthetic scene generator (shared input for the GPU library and the oracle).

This module builds geometry and kinematic scripts only: tetrahedral gel pads, closed
triangle meshes for the rigid (affine) indenters, Dirichlet flags and per-step kinematic
targets.  It contains none of the simulation method's arithmetic (no energies, no mass
properties, no contact logic); both solvers derive all of that themselves.

Conventions
-----------
* SI units (metres, kilograms, seconds, pascals).
* Soft body: ``verts`` (n,3) float64, ``tets`` (t,4) int32 with positive orientation,
  ``dirichlet`` (n,) uint8: 0 free, 1 fixed, 2 moving (prescribed each step).
* Affine body: ``verts`` (n,3) float64 world positions at creation, ``tris`` (f,3) int32,
  outward-oriented, closed.
* Body kinematic target for a step: 12 doubles ``[t0,t1,t2, A00,A01,A02,A10,...,A22]``
  meaning every creation-pose vertex X0 of that body is mapped to ``A @ X0 + t`` at the
  end of the step (the paper's kinematic constraints on the affine coordinates, Sec. 3.4 /
  App. A.5, stated in a frame that does not depend on how a solver parameterises a body).
* Moving Dirichlet targets for a step: (n_moving,3) world positions, in increasing vertex
  order of the vertices flagged 2.

Workloads (all lengths in mm in the descriptions, metres in the arrays):
* ``pad_press_cube(seed)``: 20x20x4 mm pad, Kuhn-split 8x8x2 hex grid (243 verts, 768 tets),
  bottom fixed; a 10 mm cube offset U(-2,2) mm in x,y from ``default_rng(seed)``, bottom
  0.05 mm above the pad, lowered 0.05 mm per step for 10 steps, h = 0.01 s.
* ``pad_press_slide_hull(seed)``: 32x24x6 mm pad on a 32x24x6 grid (5,775 verts,
  27,648 tets), a 400-point random convex hull (796 tris) of 8 mm extent, 0.05 mm gap,
  pressed 1.0 mm over 50 steps then slid 2.0 mm in x over 50 steps, h = 0.005 s.
* ``uniform_batch(n)``: n copies of the 8x8x2 pad, scene i from ``default_rng(1000+i)`` with
  an 8-point hull (12 tris) of 10 mm extent, xy offset U(-3,3) mm, press depth
  U(0.3,1.2) mm reached over 10 steps after closing the 0.05 mm gap.
* ``serving_request(i)`` / ``serving_arrivals(rate, duration)``: a stream of rollout requests.
  Request i (from ``default_rng([7, i])``) is the 32x24x6 mm pad on a grid drawn from
  {16x12x4, 32x24x6, 48x36x8}, with 1-3 rigid hull indenters of 8 mm extent whose triangle
  counts are log-uniform in [200, 8000] (even; n = tris/2 + 2 hull points), placed at
  non-overlapping xy positions 0.05 mm above the pad; each is pressed U(0.3,1.2) mm over 25
  steps, then all slide together U(0,2) mm in one random tangent direction over 25 steps,
  h = 0.005 s.  Arrival times are Poisson (exponential gaps from ``default_rng(seed)``).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np

MM = 1e-3

# Material and contact constants of the pad workloads (E, nu, rho of the gel; rho of the
# indenter; barrier activation distance and stiffness; Newton tolerance).
GEL_E = 0.3e6
GEL_NU = 0.45
GEL_RHO = 1000.0
ABD_RHO = 2000.0
DHAT = 1e-4
KAPPA = 1e3
KAPPA_S = 1e8
NEWTON_TOL = 1e-6


@dataclass
class BodySpec:
    verts: np.ndarray
    tris: np.ndarray
    density: float = ABD_RHO
    prescribed: bool = True


@dataclass
class SceneSpec:
    name: str
    verts: np.ndarray
    tets: np.ndarray
    dirichlet: np.ndarray
    youngs: float
    poisson: float
    density: float
    bodies: list
    params: dict
    body_targets: np.ndarray          # (n_steps, n_bodies, 12)
    dirichlet_targets: np.ndarray     # (n_steps, n_moving, 3)
    meta: dict = field(default_factory=dict)

    @property
    def n_steps(self) -> int:
        return int(self.body_targets.shape[0])


def default_params(h: float) -> dict:
    return dict(h=h, dhat=DHAT, kappa=KAPPA, kappa_s=KAPPA_S, newton_tol=NEWTON_TOL,
                gravity=(0.0, 0.0, -9.81), max_newton=100, max_al=30, max_pcg=10000,
                pcg_eta=1e-4, friction=0.0, eps_v=1e-3)


# ----------------------------------------------------------------------------- meshes
_KUHN_CACHE = {}


def kuhn_box(lo, hi, cells):
    """Cached front of ``_kuhn_box`` (returns fresh copies)."""
    key = (tuple(float(v) for v in lo), tuple(float(v) for v in hi), tuple(int(c) for c in cells))
    if key not in _KUHN_CACHE:
        _KUHN_CACHE[key] = _kuhn_box(lo, hi, cells)
    v, t = _KUHN_CACHE[key]
    return v.copy(), t.copy()


def _kuhn_box(lo, hi, cells):
    """Box [lo,hi] on an (nx,ny,nz) hex grid, each hex split into the 6 Kuhn tetrahedra.

    Vertex id = i + (nx+1)*(j + (ny+1)*k).  Cells are visited with i fastest, then j, k;
    inside a cell one tet per permutation of the axes (lexicographic order), following the
    monotone path corner -> +e_a -> +e_b -> +e_c.  Tets with negative volume get their
    second and third vertices swapped.
    """
    nx, ny, nz = cells
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    xs = [np.linspace(lo[a], hi[a], c + 1) for a, c in enumerate(cells)]
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                             indexing="ij")
    verts = np.stack([xs[0][ii.ravel()], xs[1][jj.ravel()], xs[2][kk.ravel()]], axis=1)

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    unit = np.eye(3, dtype=np.int64)
    tets = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for perm in permutations(range(3)):
                    c = np.array([i, j, k])
                    path = [c.copy()]
                    for a in perm:
                        c = c + unit[a]
                        path.append(c.copy())
                    t = [vid(*p) for p in path]
                    p0, p1, p2, p3 = (verts[q] for q in t)
                    if np.linalg.det(np.stack([p1 - p0, p2 - p0, p3 - p0], axis=1)) < 0:
                        t[1], t[2] = t[2], t[1]
                    tets.append(t)
    return verts, np.asarray(tets, dtype=np.int32)


def box_mesh(center, size):
    """Closed, outward-oriented axis-aligned box surface: 8 verts, 12 tris."""
    c = np.asarray(center, dtype=np.float64)
    h = 0.5 * np.asarray(size, dtype=np.float64)
    signs = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                      [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
    verts = c + signs * h
    tris = np.array([[0, 2, 1], [0, 3, 2],      # bottom (-z)
                     [4, 5, 6], [4, 6, 7],      # top (+z)
                     [0, 1, 5], [0, 5, 4],      # -y
                     [1, 2, 6], [1, 6, 5],      # +x
                     [2, 3, 7], [2, 7, 6],      # +y
                     [3, 0, 4], [3, 4, 7]],     # -x
                    dtype=np.int32)
    return verts, tris


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _orient_outward(verts, tris):
    c = verts.mean(axis=0)
    out = tris.copy()
    a, b, d = verts[out[:, 0]], verts[out[:, 1]], verts[out[:, 2]]
    n = np.cross(b - a, d - a)
    flip = np.einsum("ij,ij->i", n, (a + b + d) / 3.0 - c) < 0
    out[flip, 1], out[flip, 2] = tris[flip, 2], tris[flip, 1]
    return out


def random_hull(rng, n_points, extent):
    """n Gaussian directions projected onto a random ellipsoid (semi-axes U(0.6,1)), randomly
    rotated, scaled so the largest axis-aligned extent equals ``extent``; closed convex-hull
    triangulation (every point is a hull vertex, so 2n-4 tris), outward oriented, centred at
    the origin of its bounding box."""
    from scipy.spatial import ConvexHull

    d = rng.standard_normal((n_points, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    axes = rng.uniform(0.6, 1.0, size=3)
    pts = (d * axes) @ _random_rotation(rng).T
    span = pts.max(axis=0) - pts.min(axis=0)
    pts *= extent / span.max()
    pts -= 0.5 * (pts.max(axis=0) + pts.min(axis=0))
    hull = ConvexHull(pts)
    used = np.unique(hull.simplices)
    remap = -np.ones(n_points, dtype=np.int64)
    remap[used] = np.arange(len(used))
    verts = pts[used]
    tris = remap[hull.simplices].astype(np.int32)
    return verts, _orient_outward(verts, tris)


def translation_targets(offsets):
    """(n_steps, 3) translations -> (n_steps, 12) targets with A = I."""
    offsets = np.asarray(offsets, dtype=np.float64)
    out = np.zeros((len(offsets), 12))
    out[:, 0:3] = offsets
    out[:, 3:12] = np.eye(3).ravel()
    return out


def _pad_scene(name, pad_lo, pad_hi, cells, bodies, body_targets, h, meta):
    verts, tets = kuhn_box(pad_lo, pad_hi, cells)
    dirichlet = np.zeros(len(verts), dtype=np.uint8)
    dirichlet[verts[:, 2] == pad_lo[2]] = 1
    n_steps = body_targets.shape[0]
    return SceneSpec(name=name, verts=verts, tets=tets, dirichlet=dirichlet,
                     youngs=GEL_E, poisson=GEL_NU, density=GEL_RHO, bodies=bodies,
                     params=default_params(h), body_targets=body_targets,
                     dirichlet_targets=np.zeros((n_steps, 0, 3)), meta=meta)


# ----------------------------------------------------------------------------- workloads
def pad_press_cube(seed: int = 0, n_steps: int = 10) -> SceneSpec:
    rng = np.random.default_rng(seed)
    ox, oy = rng.uniform(-2.0, 2.0, size=2) * MM
    pad_lo = (-10 * MM, -10 * MM, 0.0)
    pad_hi = (10 * MM, 10 * MM, 4 * MM)
    gap = 0.05 * MM
    cube_v, cube_t = box_mesh((ox, oy, pad_hi[2] + gap + 5 * MM), (10 * MM,) * 3)
    steps = np.arange(1, n_steps + 1)
    tg = translation_targets(np.stack([0 * steps, 0 * steps, -0.05 * MM * steps], axis=1))
    return _pad_scene(f"pad_press_cube(seed={seed})", pad_lo, pad_hi, (8, 8, 2),
                      [BodySpec(cube_v, cube_t)], tg[:, None, :], 0.01,
                      dict(seed=seed, offset=(ox, oy)))


def pad_press_slide_hull(seed: int = 0, n_steps: int = 100, cells=(32, 24, 6),
                         n_points: int = 400) -> SceneSpec:
    rng = np.random.default_rng(seed)
    pad_lo = (-16 * MM, -12 * MM, 0.0)
    pad_hi = (16 * MM, 12 * MM, 6 * MM)
    gap = 0.05 * MM
    hv, ht = random_hull(rng, n_points, 8 * MM)
    hv = hv + np.array([0.0, 0.0, pad_hi[2] + gap - hv[:, 2].min()])
    off = np.zeros((n_steps, 3))
    for s in range(1, n_steps + 1):
        press = min(s, 50) / 50.0 * 1.0 * MM
        slide = max(0, s - 50) / 50.0 * 2.0 * MM
        off[s - 1] = (slide, 0.0, -press)
    return _pad_scene(f"pad_press_slide_hull(seed={seed})", pad_lo, pad_hi, cells,
                      [BodySpec(hv, ht)], translation_targets(off)[:, None, :], 0.005,
                      dict(seed=seed))


def pad_push_moving(seed: int = 0, n_steps: int = 10, rise: float = 0.04 * MM) -> SceneSpec:
    """The 8x8x2 pad with its bottom face prescribed (moving Dirichlet vertices) and raised
    by `rise` per step against a cube held in place 0.05 mm above the pad."""
    rng = np.random.default_rng(seed)
    ox, oy = rng.uniform(-2.0, 2.0, size=2) * MM
    pad_lo = (-10 * MM, -10 * MM, 0.0)
    pad_hi = (10 * MM, 10 * MM, 4 * MM)
    gap = 0.05 * MM
    cube_v, cube_t = box_mesh((ox, oy, pad_hi[2] + gap + 5 * MM), (10 * MM,) * 3)
    spec = _pad_scene(f"pad_push_moving(seed={seed})", pad_lo, pad_hi, (8, 8, 2),
                      [BodySpec(cube_v, cube_t)], translation_targets(np.zeros((n_steps, 3)))[:, None, :],
                      0.01, dict(seed=seed, offset=(ox, oy), rise=rise))
    bottom = spec.dirichlet == 1
    spec.dirichlet[bottom] = 2
    base = spec.verts[bottom]
    steps = np.arange(1, n_steps + 1)
    spec.dirichlet_targets = base[None, :, :] + np.array([0.0, 0.0, 1.0])[None, None, :] * (rise * steps)[:, None, None]
    return spec


def pad_press_slide_friction(seed: int = 0, n_steps: int = 8, mu: float = 0.5,
                             eps_v: float = 1e-3) -> SceneSpec:
    """The 8x8x2 pad and the 10 mm cube with friction: the cube closes the 0.05 mm gap and
    presses 0.15 mm over the first half of the steps, then slides 0.1 mm per step in x."""
    rng = np.random.default_rng(seed)
    ox, oy = rng.uniform(-2.0, 2.0, size=2) * MM
    pad_lo = (-10 * MM, -10 * MM, 0.0)
    pad_hi = (10 * MM, 10 * MM, 4 * MM)
    cube_v, cube_t = box_mesh((ox, oy, pad_hi[2] + 0.05 * MM + 5 * MM), (10 * MM,) * 3)
    half = n_steps // 2
    k = np.arange(1, n_steps + 1)
    dz = -0.05 * MM * np.minimum(k, half)
    dx = 0.1 * MM * np.maximum(k - half, 0)
    tg = translation_targets(np.stack([dx, 0 * dx, dz], axis=1))
    spec = _pad_scene(f"pad_press_slide_friction(seed={seed})", pad_lo, pad_hi, (8, 8, 2),
                      [BodySpec(cube_v, cube_t)], tg[:, None, :], 0.01,
                      dict(seed=seed, offset=(ox, oy), mu=mu, eps_v=eps_v))
    spec.params["friction"] = mu
    spec.params["eps_v"] = eps_v
    return spec


def cube_resting_on_pad(mu: float = 0.1, n_steps: int = 30, eps_v: float = 1e-3) -> SceneSpec:
    """A free (unprescribed) 10 mm cube released 0.05 mm above the centre of the 8x8x2 pad,
    under gravity, with friction coefficient mu; h = 0.01 s."""
    pad_lo = (-10 * MM, -10 * MM, 0.0)
    pad_hi = (10 * MM, 10 * MM, 4 * MM)
    cube_v, cube_t = box_mesh((0.0, 0.0, pad_hi[2] + 0.05 * MM + 5 * MM), (10 * MM,) * 3)
    hold = translation_targets(np.zeros((n_steps, 3)))[:, None, :]  # unused: the cube is free
    spec = _pad_scene("cube_resting_on_pad", pad_lo, pad_hi, (8, 8, 2),
                      [BodySpec(cube_v, cube_t, prescribed=False)], hold, 0.01,
                      dict(mu=mu, eps_v=eps_v))
    spec.params["friction"] = mu
    spec.params["eps_v"] = eps_v
    return spec


def top_surface_tris(spec: SceneSpec) -> np.ndarray:
    """Boundary triangles of the pad's top face (the coated, contact side), outward (+z)
    oriented, in the order their tets appear: (f, 3) int32 soft-vertex ids."""
    zt = spec.verts[:, 2].max()
    count = {}
    faces = []
    for t in spec.tets:
        for drop in range(4):
            f = [int(v) for k, v in enumerate(t) if k != drop]
            key = tuple(sorted(f))
            count[key] = count.get(key, 0) + 1
            faces.append((key, f))
    out = []
    for key, f in faces:
        if count[key] != 1 or not np.all(spec.verts[f, 2] == zt):
            continue
        a, b, c = spec.verts[f]
        if np.cross(b - a, c - a)[2] < 0:
            f = [f[0], f[2], f[1]]
        out.append(f)
    return np.asarray(out, dtype=np.int32)


def marker_layout(spec: SceneSpec, tris: np.ndarray, nx: int, ny: int, margin: float = 1.5 * MM):
    """A regular nx-by-ny grid of markers on the top face (inset by ``margin``), each given as
    the first of ``tris`` whose rest projection contains it and its barycentric coordinates:
    (tri index into ``tris`` (m,), barycentric (m, 3))."""
    lo = spec.verts[:, :2].min(0) + margin
    hi = spec.verts[:, :2].max(0) - margin
    gx, gy = np.meshgrid(np.linspace(lo[0], hi[0], nx), np.linspace(lo[1], hi[1], ny))
    pts = np.stack([gx.ravel(), gy.ravel()], axis=1)
    P = spec.verts[tris][:, :, :2]
    idx, bary = [], []
    for q in pts:
        a, b, c = P[:, 0], P[:, 1], P[:, 2]
        den = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
        l1 = ((q[0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (q[1] - a[:, 1])) / den
        l2 = ((b[:, 0] - a[:, 0]) * (q[1] - a[:, 1]) - (q[0] - a[:, 0]) * (b[:, 1] - a[:, 1])) / den
        inside = np.flatnonzero((l1 >= 0) & (l2 >= 0) & (l1 + l2 <= 1))
        k = int(inside[0])
        idx.append(k)
        b = np.maximum([1.0 - l1[k] - l2[k], l1[k], l2[k]], 0.0)
        bary.append(b / b.sum())
    return np.asarray(idx, dtype=np.int32), np.asarray(bary, dtype=np.float64)


def batch_member(i: int, n_steps: int = 10) -> SceneSpec:
    rng = np.random.default_rng(1000 + i)
    pad_lo = (-10 * MM, -10 * MM, 0.0)
    pad_hi = (10 * MM, 10 * MM, 4 * MM)
    gap = 0.05 * MM
    hv, ht = random_hull(rng, 8, 10 * MM)
    ox, oy = rng.uniform(-3.0, 3.0, size=2) * MM
    depth = rng.uniform(0.3, 1.2) * MM
    hv = hv + np.array([ox, oy, pad_hi[2] + gap - hv[:, 2].min()])
    steps = np.arange(1, n_steps + 1)
    dz = -(depth + gap) * steps / n_steps
    tg = translation_targets(np.stack([0 * dz, 0 * dz, dz], axis=1))
    return _pad_scene(f"uniform_batch[{i}]", pad_lo, pad_hi, (8, 8, 2),
                      [BodySpec(hv, ht)], tg[:, None, :], 0.01,
                      dict(index=i, offset=(ox, oy), depth=depth))


SERVING_GRIDS = ((16, 12, 4), (32, 24, 6), (48, 36, 8))


def serving_request(i: int, n_press: int = 25, n_slide: int = 25) -> SceneSpec:
    rng = np.random.default_rng([7, i])
    pad_lo = (-16 * MM, -12 * MM, 0.0)
    pad_hi = (16 * MM, 12 * MM, 6 * MM)
    gap = 0.05 * MM
    cells = SERVING_GRIDS[int(rng.integers(len(SERVING_GRIDS)))]
    n_bodies = int(rng.integers(1, 4))
    # xy centres at least 9 mm apart along some axis (the 8 mm hull boxes never overlap,
    # and they slide together)
    centres = []
    for _ in range(1000):
        if len(centres) == n_bodies:
            break
        c = rng.uniform((-10 * MM, -6 * MM), (10 * MM, 6 * MM))
        if all(max(abs(c[0] - o[0]), abs(c[1] - o[1])) >= 9 * MM for o in centres):
            centres.append(c)
    n_steps = n_press + n_slide
    ang = rng.uniform(0.0, 2.0 * np.pi)
    slide = rng.uniform(0.0, 2.0) * MM * np.array([np.cos(ang), np.sin(ang)])
    bodies, targets = [], []
    for c in centres:
        tris = 2 * int(round(0.5 * np.exp(rng.uniform(np.log(200.0), np.log(8000.0)))))
        hv, ht = random_hull(rng, tris // 2 + 2, 8 * MM)
        hv = hv + np.array([c[0], c[1], pad_hi[2] + gap - hv[:, 2].min()])
        depth = rng.uniform(0.3, 1.2) * MM
        off = np.zeros((n_steps, 3))
        for s in range(1, n_steps + 1):
            off[s - 1, 2] = -(depth + gap) * min(s, n_press) / n_press
            off[s - 1, :2] = slide * max(0, s - n_press) / n_slide
        bodies.append(BodySpec(hv, ht))
        targets.append(translation_targets(off))
    return _pad_scene(f"serving_request[{i}]", pad_lo, pad_hi, cells, bodies,
                      np.stack(targets, axis=1), 0.005,
                      dict(index=i, cells=cells, n_bodies=len(bodies),
                           tris=[len(b.tris) for b in bodies]))


def serving_arrivals(rate: float, duration: float, seed: int = 7) -> np.ndarray:
    """Poisson arrival times (s) in [0, duration) at the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)


def uniform_batch(n: int = 256, n_steps: int = 10):
    return [batch_member(i, n_steps) for i in range(n)]


def apply_target(X0: np.ndarray, q: np.ndarray) -> np.ndarray:
    """World positions of creation-pose vertices X0 under a 12-double target q."""
    A = np.asarray(q[3:12]).reshape(3, 3)
    return X0 @ A.T + np.asarray(q[0:3])


# ----------------------------------------------------------------------------- robot-driven scenes
def _trans(t):
    T = np.eye(4)
    T[:3, 3] = t
    return T


def _rot_z(angle):
    c, s = np.cos(angle), np.sin(angle)
    T = np.eye(4)
    T[:2, :2] = [[c, -s], [s, c]]
    return T


def _apply(T, pts):
    return pts @ T[:3, :3].T + T[:3, 3]


def parallel_gripper_fk(base_z: float, opening: float, mount1=(0.0, 0.0, 0.0)):
    """Forward kinematics of a parallel-jaw gripper: a base link on a prismatic joint along z
    (joint value base_z) carrying two fingers on prismatic joints along x, each opening/2
    from the base axis.  Finger 0 (at -x) keeps the base orientation, so its local +x points
    to the other finger; finger 1 is turned by pi about z and mounted at the fixed offset
    mount1 in its own frame.  Returns the 4x4 world transforms of the two finger links."""
    base = _trans((0.0, 0.0, base_z))
    left = base @ _trans((-0.5 * opening, 0.0, 0.0))
    right = base @ _trans((0.5 * opening, 0.0, 0.0)) @ _rot_z(np.pi) @ _trans(mount1)
    return left, right


def _link_target(T_now, T_rest):
    """Body target (t, A row-major) moving a link's creation-pose vertices with the link."""
    M = T_now @ np.linalg.inv(T_rest)
    out = np.zeros(12)
    out[0:3] = M[:3, 3]
    out[3:12] = M[:3, :3].ravel()
    return out


def gripper_scene(name, obj, joint_traj, h, cells=(6, 32, 24), pad_size=(6 * MM, 32 * MM, 24 * MM),
                  link_gap=0.2 * MM, plate=3.0 * MM, friction=0.0, gravity=(0.0, 0.0, 0.0),
                  mount1=(0.0, 0.0, 0.0), meta=None):
    """A gel pad on each finger of the parallel gripper (Sec. 4.1: a sensor's gel is a tet mesh
    attached to a robot link by its back face), an optional free object, and a script of
    joint values turned into kinematic targets by forward kinematics.

    In a finger's frame the pad fills [0, t] x [-w/2, w/2] x [-d/2, d/2] (pad_size (t, w, d),
    hex cells `cells` along (x, y, z)); its back face x = 0 is attached to the link (moving
    Dirichlet vertices that follow the link), its coated face x = t faces the other finger.
    mount1 offsets finger 1 in its own frame (see parallel_gripper_fk).
    The link itself is a rigid plate behind the pad, link_gap away (more than dhat), driven
    as a prescribed affine body.  joint_traj: (n_steps + 1, 2) rows (base_z, opening), row 0
    the creation pose, row k the targets at the end of step k.  Soft vertices: finger 0's pad,
    then finger 1's.  Bodies: the object (free) if given, then the two links."""
    t, w, d = pad_size
    pv, pt = kuhn_box((0.0, -0.5 * w, -0.5 * d), (t, 0.5 * w, 0.5 * d), cells)
    lv, lt = box_mesh((-link_gap - 0.5 * plate, 0.0, 0.0), (plate, w, d))
    T0 = parallel_gripper_fk(*joint_traj[0], mount1=mount1)
    verts = np.concatenate([_apply(T0[0], pv), _apply(T0[1], pv)])
    tets = np.concatenate([pt, pt + len(pv)]).astype(np.int32)
    back = np.where(pv[:, 0] == 0.0)[0]
    dirichlet = np.zeros(len(verts), dtype=np.uint8)
    dirichlet[back] = 2
    dirichlet[back + len(pv)] = 2
    n_steps = len(joint_traj) - 1
    moving = np.concatenate([back, back + len(pv)])
    dir_t = np.zeros((n_steps, len(moving), 3))
    links = [BodySpec(_apply(T0[f], lv), lt.copy(), prescribed=True) for f in range(2)]
    bodies = ([BodySpec(obj[0], obj[1], prescribed=False)] if obj is not None else []) + links
    body_t = np.zeros((n_steps, len(bodies), 12))
    body_t[:, :, 3:12] = np.eye(3).ravel()
    for k in range(1, n_steps + 1):
        Tk = parallel_gripper_fk(*joint_traj[k], mount1=mount1)
        dir_t[k - 1] = np.concatenate([_apply(Tk[0], pv[back]), _apply(Tk[1], pv[back])])
        for f in range(2):
            body_t[k - 1, len(bodies) - 2 + f] = _link_target(Tk[f], T0[f])
    params = default_params(h)
    params["gravity"] = tuple(gravity)
    params["friction"] = friction
    return SceneSpec(name=name, verts=verts, tets=tets, dirichlet=dirichlet, youngs=GEL_E,
                     poisson=GEL_NU, density=GEL_RHO, bodies=bodies, params=params,
                     body_targets=body_t, dirichlet_targets=dir_t,
                     meta=dict(meta or {}, joint_traj=np.asarray(joint_traj), pad_vertices=len(pv),
                               mount1=tuple(mount1)))


def grasp_lift(seed: int = 0, cells=(6, 32, 24), n_points: int = 5002, extent: float = 24 * MM,
               n_squeeze: int = 20, n_lift: int = 180, squeeze: float = 0.5 * MM,
               lift: float = 20 * MM, gap: float = 0.05 * MM, friction: float = 0.5,
               h: float = 0.005) -> SceneSpec:
    """Two-finger grasp: a free object (a random convex hull of n_points, extent 24 mm, from
    default_rng(5000 + seed)) between the two pads of the parallel gripper, their coated faces
    `gap` from it.  The fingers close by gap + squeeze each over n_squeeze steps, then the
    base rises by `lift` over n_lift steps.  The pads hold the object by friction (Coulomb
    coefficient `friction`, App. A.3) against gravity; friction = 0 turns gravity off too (a
    frictionless squeeze of an irregular object is not a grasp: it spins or squirts out)."""
    rng = np.random.default_rng(5000 + seed)
    hv, ht = random_hull(rng, n_points, extent)
    half = 0.5 * (hv[:, 0].max() - hv[:, 0].min())
    hv = hv - np.array([0.5 * (hv[:, 0].max() + hv[:, 0].min()), 0.0, 0.0])
    t = 6 * MM
    open0 = 2.0 * (t + half + gap)
    traj = [(0.0, open0)]
    for k in range(1, n_squeeze + n_lift + 1):
        close = min(k, n_squeeze) / n_squeeze * 2.0 * (gap + squeeze)
        rise = max(0, k - n_squeeze) / n_lift * lift
        traj.append((rise, open0 - close))
    grav = (0.0, 0.0, -9.81) if friction > 0.0 else (0.0, 0.0, 0.0)
    return gripper_scene(f"grasp_lift(seed={seed})", (hv, ht), np.array(traj), h, cells=cells,
                         friction=friction, gravity=grav,
                         meta=dict(seed=seed, object_tris=len(ht), half_width=half))
