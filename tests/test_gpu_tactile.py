"""GPU parity of the tactile outputs (Taccel Sec. 4.2) through the C-ABI: marker positions and
flows and depth maps bit for bit equal to the oracle's definitions on the same state (the
coverage and depth arithmetic is FMA-free FP64 on both sides), normal maps within 1e-15."""
import numpy as np
import pytest

from oracle import tactile as TO
from paper_2504_12908_amd import scenes as S

pytestmark = pytest.mark.gpu
MM = S.MM


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def T():
    from paper_2504_12908_amd import taccel
    taccel.lib()
    return taccel


@pytest.fixture(scope="module")
def pressed(T):
    """The small pad after three steps of the cube press (GPU state)."""
    spec = S.pad_press_cube(0)
    g = T.Scene(spec)
    for k in range(3):
        rc, _ = g.step(k)
        assert rc == T.OK
    x = g.read(T.FIELD_X)
    yield spec, g, x
    g.close()


def _cams():
    th, tilt = 0.3, 0.1
    eu = np.array([np.cos(th), np.sin(th), 0.0])
    ev = np.array([-np.sin(th) * np.cos(tilt), np.cos(th) * np.cos(tilt), np.sin(tilt)])
    return [
        dict(origin=(-11 * MM, -11 * MM, 0.0), eu=(1.0, 0.0, 0.0), ev=(0.0, 1.0, 0.0),
             pixel=0.35 * MM, width=64, height=64),
        dict(origin=(-13 * MM, 9 * MM, 9 * MM), eu=tuple(eu), ev=tuple(-ev), pixel=0.3 * MM,
             width=72, height=80),
    ]


def test_markers_parity(T, pressed):
    spec, g, x = pressed
    tris = S.top_surface_tris(spec)
    idx, bary = S.marker_layout(spec, tris, 9, 9)
    say(f"markers: {len(idx)} on {spec.name} after 3 steps")
    pos, flow = g.markers(tris[idx], bary)
    po, fo = TO.markers(x, spec.verts, tris[idx], bary)
    assert np.array_equal(pos, po) and np.array_equal(flow, fo)
    assert np.abs(flow[:, 2]).max() > 1e-5  # the press shows in the flow


@pytest.mark.parametrize("which", [0, 1])
def test_depth_map_parity(T, pressed, which):
    spec, g, x = pressed
    tris = S.top_surface_tris(spec)
    c = _cams()[which]
    say(f"depth map {c['width']}x{c['height']} camera {which} on {spec.name}")
    cam = T.camera(c["origin"], c["eu"], c["ev"], c["pixel"], c["width"], c["height"])
    depth, normal = g.depth_map(cam, tris)
    do, no = TO.depth_map(x, tris, c["origin"], c["eu"], c["ev"], c["pixel"], c["width"],
                          c["height"])
    cov = np.isfinite(do)
    assert np.array_equal(np.isfinite(depth), cov)
    assert np.array_equal(depth[cov], do[cov])
    assert np.abs(normal - no).max() <= 1e-15
    assert cov.sum() > 0.5 * cov.size
    assert np.all(normal[~cov] == 0.0)
    if which == 0:  # the press dents the face: some depths below 4 mm
        assert depth[cov].min() < 4 * MM - 1e-5


def test_depth_map_full_size_sampled(T):
    """The benchmark pad (1,536 coated-face triangles) after two steps, a 640x480 map at 50 um
    over the whole face: every pixel covered; 600 sampled pixels equal to the oracle's."""
    spec = S.pad_press_slide_hull(0)
    g = T.Scene(spec)
    for k in range(2):
        assert g.step(k)[0] == T.OK
    x = g.read(T.FIELD_X)
    tris = S.top_surface_tris(spec)
    c = dict(origin=(-16 * MM, -12 * MM, 0.0), eu=(1.0, 0.0, 0.0), ev=(0.0, 1.0, 0.0),
             pixel=0.05 * MM, width=640, height=480)
    say("depth map 640x480 on the 5,775-vertex pad")
    cam = T.camera(c["origin"], c["eu"], c["ev"], c["pixel"], c["width"], c["height"])
    depth, normal = g.depth_map(cam, tris)
    g.close()
    assert np.all(np.isfinite(depth))
    rng = np.random.default_rng(11)
    pix = [(int(i), int(j)) for i, j in zip(rng.integers(0, 480, 560), rng.integers(0, 640, 560))]
    pix += [(0, 0), (0, 639), (479, 0), (479, 639)] + [(240, j) for j in range(300, 336)]
    do, no = TO.depth_map(x, tris, c["origin"], c["eu"], c["ev"], c["pixel"], 640, 480, pixels=pix)
    ii = np.array([p[0] for p in pix])
    jj = np.array([p[1] for p in pix])
    assert np.array_equal(depth[ii, jj], do)
    assert np.abs(normal[ii, jj] - no).max() <= 1e-15


def test_batch_tactile_equals_scene(T):
    specs = [S.batch_member(0), S.batch_member(1)]
    b = T.Batch(specs)
    s1 = T.Scene(specs[1])
    assert b.step(0)[0] == T.OK and s1.step(0)[0] == T.OK
    tris = S.top_surface_tris(specs[1])
    idx, bary = S.marker_layout(specs[1], tris, 5, 5)
    c = _cams()[0]
    cam = T.camera(c["origin"], c["eu"], c["ev"], c["pixel"], c["width"], c["height"])
    assert all(np.array_equal(a, b_) for a, b_ in zip(b.markers(1, tris[idx], bary),
                                                       s1.markers(tris[idx], bary)))
    db, nb = b.depth_map(1, cam, tris)
    ds, ns = s1.depth_map(cam, tris)
    assert np.array_equal(db, ds) and np.array_equal(nb, ns)
    b.close()
    s1.close()


def test_tactile_argument_errors(T, pressed):
    spec, g, x = pressed
    tris = S.top_surface_tris(spec)
    bad = T.camera((0, 0, 0), (1.0, 0.0, 0.0), (0.5, 0.5, 0.0), 1e-4, 8, 8)
    with pytest.raises(T.TaccelError):
        g.depth_map(bad, tris)
    with pytest.raises(T.TaccelError):
        g.depth_map(T.camera((0, 0, 0), (1.0, 0, 0), (0, 1.0, 0), 1e-4, 0, 8), tris)
    with pytest.raises(T.TaccelError):
        g.markers(np.array([[0, 1, len(spec.verts)]]), np.array([[0.2, 0.3, 0.5]]))
    with pytest.raises(T.TaccelError):
        g.markers(tris[:1], np.array([[1.2, -0.1, -0.1]]))
