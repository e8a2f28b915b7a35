"""Pins of the tactile-output oracle (markers, depth and normal maps; Taccel Sec. 4.2) against
closed forms: rest and rigid-motion flows, flat and tilted surfaces, coverage of a
rectangle, the nearer of two surfaces."""
import math

import numpy as np
import pytest

from oracle import tactile as TO
from paper_2504_12908_amd import scenes as S

MM = S.MM


@pytest.fixture(scope="module")
def pad():
    spec = S.pad_press_cube(0)
    tris = S.top_surface_tris(spec)
    return spec, tris


def test_top_surface_and_markers_layout(pad):
    spec, tris = pad
    assert tris.shape == (128, 3)  # 8x8 cells, two triangles each
    P = spec.verts[tris]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    assert np.all(n[:, 2] > 0) and np.allclose(n[:, :2], 0)
    assert np.isclose(0.5 * n[:, 2].sum(), (20 * MM) ** 2, rtol=1e-12)  # covers the face once
    idx, bary = S.marker_layout(spec, tris, 7, 7)
    assert np.all(bary >= 0) and np.allclose(bary.sum(1), 1.0, rtol=0, atol=1e-15)


def test_markers_rest_rigid_and_vertices(pad):
    spec, tris = pad
    idx, bary = S.marker_layout(spec, tris, 7, 7)
    X = spec.verts
    pos, flow = TO.markers(X, X, tris[idx], bary)
    assert np.all(flow == 0.0)
    assert np.allclose(pos[:, 2], 4 * MM, rtol=0, atol=1e-18)
    d = np.array([1.5e-4, -2.5e-4, 3e-5])
    pos2, flow2 = TO.markers(X + d, X, tris[idx], bary)
    assert np.allclose(flow2, d, rtol=0, atol=2e-17)  # rounding of positions ~1e-2 m
    # a marker at a vertex follows that vertex exactly
    e = np.eye(3)[[0, 1, 2]]
    rng = np.random.default_rng(5)
    x = X + rng.normal(size=X.shape) * 1e-4
    pos3, _ = TO.markers(x, X, tris[:3], e)
    assert np.array_equal(pos3, x[tris[np.arange(3), np.arange(3)]])


def _below(width_px, height_px, pix, z0=0.0):
    # image plane at height z0 under the pad, looking up (+z), covering [-12, 12]^2 mm
    return dict(origin=(-12 * MM, -12 * MM, z0), eu=(1.0, 0.0, 0.0), ev=(0.0, 1.0, 0.0),
                pixel=pix, width=width_px, height=height_px)


def test_depth_flat_face_coverage_and_normals(pad):
    spec, tris = pad
    cam = _below(48, 48, 0.5 * MM)
    depth, normal = TO.depth_map(spec.verts, tris, cam["origin"], cam["eu"], cam["ev"],
                                 cam["pixel"], cam["width"], cam["height"])
    # pixel centres at -12 + (k + 1/2) 0.5 mm: inside [-10, 10] for k = 4 .. 43
    inside = np.zeros((48, 48), bool)
    inside[4:44, 4:44] = True
    assert np.array_equal(np.isfinite(depth), inside)
    assert np.allclose(depth[inside], 4 * MM, rtol=1e-15, atol=0)
    assert np.all(normal[inside] == np.array([0.0, 0.0, -1.0]))
    assert np.all(normal[~inside] == 0.0)


def test_depth_tilted_surface_closed_form(pad):
    spec, tris = pad
    x = spec.verts.copy()
    top = x[:, 2] == x[:, 2].max()
    x[top, 2] += 0.05 * x[top, 0] - 0.02 * x[top, 1]  # a plane: interpolation is exact
    cam = _below(40, 40, 0.5 * MM, z0=-1 * MM)
    depth, normal = TO.depth_map(x, tris, cam["origin"], cam["eu"], cam["ev"], cam["pixel"],
                                 cam["width"], cam["height"])
    jj, ii = np.meshgrid(np.arange(40), np.arange(40))
    u = -12 * MM + (jj + 0.5) * 0.5 * MM
    v = -12 * MM + (ii + 0.5) * 0.5 * MM
    expect = 1 * MM + 4 * MM + 0.05 * u - 0.02 * v
    ok = np.isfinite(depth)
    assert ok.sum() == 36 * 36
    assert np.allclose(depth[ok], expect[ok], rtol=1e-13, atol=0)
    nz = np.array([-0.05, 0.02, 1.0]) / math.sqrt(0.05 ** 2 + 0.02 ** 2 + 1)
    assert np.allclose(normal[ok], -nz, rtol=0, atol=1e-15)


def test_depth_picks_the_nearer_surface(pad):
    spec, tris = pad
    n = len(spec.verts)
    x2 = np.vstack([spec.verts, spec.verts - np.array([0, 0, 1 * MM])])  # second copy lower
    tris2 = np.vstack([tris, tris + n])
    cam = _below(24, 24, 1 * MM)
    d1, _ = TO.depth_map(x2, tris2, cam["origin"], cam["eu"], cam["ev"], cam["pixel"], 24, 24)
    assert np.allclose(d1[np.isfinite(d1)], 3 * MM, rtol=1e-15, atol=0)
    # looking down from above (e_n = -z) the upper copy is the nearer one
    above = dict(origin=(-12 * MM, 12 * MM, 10 * MM), eu=(1.0, 0.0, 0.0), ev=(0.0, -1.0, 0.0))
    d2, n2 = TO.depth_map(x2, tris2, above["origin"], above["eu"], above["ev"], 1 * MM, 24, 24)
    ok = np.isfinite(d2)
    assert np.allclose(d2[ok], 6 * MM, rtol=1e-15, atol=0)
    assert np.all(n2[ok] == np.array([0.0, 0.0, 1.0]))
