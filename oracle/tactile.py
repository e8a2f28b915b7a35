"""Tactile outputs of a deformed gel pad, written out from their definitions (Taccel Sec. 4.2).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import this module; the GPU library never does.

* Markers: a marker sits on a surface triangle at fixed barycentric coordinates; its
  position is the same combination of the triangle's current vertex positions, and its flow
  is that position minus the one of the rest configuration.
* Depth and normal maps: the deformed coated surface (a triangle list) seen orthographically
  from an image plane.  Pixel (i, j) is the ray from origin + (j + 1/2) p e_u + (i + 1/2) p e_v
  along e_n = e_u x e_v.  A triangle covers the pixel when the pixel centre lies in its
  projection onto the plane (edges included); the depth is the smallest ray parameter over
  the covering triangles (ties: the lowest triangle index), +inf where none covers; the
  normal is that triangle's unit normal turned towards the image plane, zero where none.

Every floating-point expression is evaluated in the order written (plain IEEE FP64 numpy
operations, no fused multiply-add), the order the GPU path uses too, so pixel coverage
decisions are reproducible bit for bit.
"""
from __future__ import annotations

import math

import numpy as np


def markers(x, X, tris, bary):
    """Positions (m, 3) and flows (m, 3) of markers on triangles ``tris`` (m, 3) of soft-vertex
    ids with barycentric coordinates ``bary`` (m, 3); x current and X rest positions (n, 3)."""
    x = np.asarray(x, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    b = np.asarray(bary, dtype=np.float64)
    t = np.asarray(tris)
    pos = (b[:, 0:1] * x[t[:, 0]] + b[:, 1:2] * x[t[:, 1]]) + b[:, 2:3] * x[t[:, 2]]
    rest = (b[:, 0:1] * X[t[:, 0]] + b[:, 1:2] * X[t[:, 1]]) + b[:, 2:3] * X[t[:, 2]]
    return pos, pos - rest


def camera_normal(eu, ev):
    """e_n = e_u x e_v, component by component."""
    return np.array([eu[1] * ev[2] - eu[2] * ev[1],
                     eu[2] * ev[0] - eu[0] * ev[2],
                     eu[0] * ev[1] - eu[1] * ev[0]])


def _project(x, o, eu, ev, en):
    d = x - o
    u = (d[..., 0] * eu[0] + d[..., 1] * eu[1]) + d[..., 2] * eu[2]
    v = (d[..., 0] * ev[0] + d[..., 1] * ev[1]) + d[..., 2] * ev[2]
    t = (d[..., 0] * en[0] + d[..., 1] * en[1]) + d[..., 2] * en[2]
    return u, v, t


def depth_pixel(U, V, T, a, b):
    """Coverage and ray parameter of the pixel centre (a, b) for every triangle (arrays of
    projected vertex coordinates U, V (ntri, 3) and ray parameters T (ntri, 3))."""
    w0 = (U[:, 1] - a) * (V[:, 2] - b) - (U[:, 2] - a) * (V[:, 1] - b)
    w1 = (U[:, 2] - a) * (V[:, 0] - b) - (U[:, 0] - a) * (V[:, 2] - b)
    w2 = (U[:, 0] - a) * (V[:, 1] - b) - (U[:, 1] - a) * (V[:, 0] - b)
    A = (w0 + w1) + w2
    pos = (A > 0.0) & (w0 >= 0.0) & (w1 >= 0.0) & (w2 >= 0.0)
    neg = (A < 0.0) & (w0 <= 0.0) & (w1 <= 0.0) & (w2 <= 0.0)
    inside = pos | neg
    with np.errstate(divide="ignore", invalid="ignore"):
        t = ((w0 * T[:, 0] + w1 * T[:, 1]) + w2 * T[:, 2]) / A
    return inside, t


def face_normal(x, tri, en):
    """Unit normal of triangle ``tri`` at positions x, turned so that n . e_n <= 0."""
    p0, p1, p2 = x[tri[0]], x[tri[1]], x[tri[2]]
    e1 = p1 - p0
    e2 = p2 - p0
    n = np.array([e1[1] * e2[2] - e1[2] * e2[1],
                  e1[2] * e2[0] - e1[0] * e2[2],
                  e1[0] * e2[1] - e1[1] * e2[0]])
    ln = math.sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2])
    n = n / ln
    if (n[0] * en[0] + n[1] * en[1]) + n[2] * en[2] > 0.0:
        n = -n
    return n


def depth_map(x, tris, origin, eu, ev, pixel, width, height, pixels=None):
    """Depth (height, width) and normal (height, width, 3) maps, or, with ``pixels`` a list of
    (i, j), the depth (k,) and normal (k, 3) of those pixels only."""
    x = np.asarray(x, dtype=np.float64)
    tris = np.asarray(tris)
    o = np.asarray(origin, dtype=np.float64)
    eu = np.asarray(eu, dtype=np.float64)
    ev = np.asarray(ev, dtype=np.float64)
    en = camera_normal(eu, ev)
    U, V, T = _project(x[tris], o, eu, ev, en)
    full = pixels is None
    if full:
        pixels = [(i, j) for i in range(height) for j in range(width)]
    depth = np.full(len(pixels), np.inf)
    normal = np.zeros((len(pixels), 3))
    for k, (i, j) in enumerate(pixels):
        a = (j + 0.5) * pixel
        b = (i + 0.5) * pixel
        inside, t = depth_pixel(U, V, T, a, b)
        cand = np.flatnonzero(inside)
        if len(cand) == 0:
            continue
        best = cand[np.argmin(t[cand])]  # argmin returns the first (lowest index) minimum
        depth[k] = t[best]
        normal[k] = face_normal(x, tris[best], en)
    if full:
        return depth.reshape(height, width), normal.reshape(height, width, 3)
    return depth, normal
