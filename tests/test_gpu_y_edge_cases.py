"""Degenerate and ragged inputs through the C-ABI, against the oracle or against each scene
run alone: a pad with no body at all, a body far from the pad (no contact candidate, so every
pair array of the step is empty), a free body above a pad whose every vertex is fixed (no soft
unknown), a scene with nothing free at all, and a batch of scenes of very different sizes.
"""
import numpy as np
import pytest

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


def _small_pad(n_steps, bodies, body_targets, fixed_all=False):
    spec = S._pad_scene("edge", (-10 * MM, -10 * MM, 0.0), (10 * MM, 10 * MM, 4 * MM), (4, 4, 2),
                        bodies, body_targets, 0.01, {})
    if fixed_all:
        spec.dirichlet[:] = 1
    return spec


def _no_body(n=3):
    return _small_pad(n, [], np.zeros((n, 0, 12)))


def _far_body(n=3):
    cv, ct = S.box_mesh((0.0, 0.0, 30 * MM), (5 * MM,) * 3)
    return _small_pad(n, [S.BodySpec(cv, ct, prescribed=False)], np.zeros((n, 1, 12)))


def _free_body_over_fixed_pad(n=3):
    # tilted, so that it lands on a corner (a flat face landing on a flat triangulated face is
    # a degenerate contact whose frictionless tangential position is not well determined)
    cv, ct = S.box_mesh((0.0, 0.0, 0.0), (5 * MM,) * 3)
    a, b = 0.3, 0.2
    Rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    cv = cv @ (Ry @ Rx).T
    cv = cv + np.array([1.3 * MM, -0.7 * MM, 4 * MM + 0.3 * MM - cv[:, 2].min()])
    return _small_pad(n, [S.BodySpec(cv, ct, prescribed=False)], np.zeros((n, 1, 12)),
                      fixed_all=True)


@pytest.mark.parametrize("make", [_no_body, _far_body, _free_body_over_fixed_pad])
def test_degenerate_scene_teacher_forced(T, oracle_lib, make):
    spec = make()
    say(f"degenerate scene: {make.__name__}")
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec)
    L = o.scale
    for k in range(spec.n_steps):
        g.set_state(*o.get_state())
        rc_o, _ = o.step(k)
        rc_g, st = g.step(k)
        assert rc_o == 0 and rc_g == T.OK, (k, rc_o, T.STATUS_NAMES[rc_g], st)
        xo, _, qo, _ = o.get_state()
        xg, _, qg, _ = g.get_state()
        err = np.abs(xg - xo).max()
        if len(spec.bodies):
            err = max(err, np.abs(qg[:, :3] - qo[:, :3]).max())
        say(f"  step {k}: newton {st['newton_iters']} active {st['n_active']} err {err:.3e}")
        assert err <= 1e-8 * L
        assert len(g.contacts()) == st["n_active"] or k < spec.n_steps - 1


def test_nothing_free(T):
    spec = _small_pad(2, [], np.zeros((2, 0, 12)), fixed_all=True)
    g = T.Scene(spec)
    for k in range(2):
        rc, st = g.step(k)
        assert rc == T.OK, st
        assert np.array_equal(g.read(T.FIELD_X), spec.verts)
    g.close()


def test_ragged_batch_equals_single(T):
    specs = [_no_body(), S.batch_member(5, n_steps=3), _far_body(), _free_body_over_fixed_pad(),
             S.pad_press_slide_hull(3, n_steps=3, cells=(4, 4, 2), n_points=10)]
    say("ragged batch: 5 scenes of 75 to 243 vertices, 0 or 1 body, vs each alone")
    b = T.Batch(specs)
    singles = [T.Scene(s) for s in specs]
    for k in range(3):
        rc, per, st = b.step(k)
        assert rc == T.OK, per
        for i, sg in enumerate(singles):
            r, _ = sg.step(k)
            assert r == T.OK
            assert np.array_equal(b.read(i, T.FIELD_X), sg.read(T.FIELD_X))
            if specs[i].bodies:
                assert np.array_equal(b.read(i, T.FIELD_Q), sg.read(T.FIELD_Q))
    b.close()
    for sg in singles:
        sg.close()
