"""Failure isolation in a batch: a scene whose state has exploded (a surface vertex a
kilometre away, so its contact boxes span far more grid cells than any real step can) fails
with TACCEL_NAN and is rolled back, while the other scenes of the batch step exactly as they
do alone."""
import numpy as np
import pytest

from paper_2504_12908_amd import scenes as S

pytestmark = pytest.mark.gpu


def test_exploded_scene_fails_alone(T=None):
    from paper_2504_12908_amd import taccel as T
    specs = [S.batch_member(40), S.batch_member(41)]
    print("batch of 2, scene 1 with a vertex moved 1 km up", flush=True)
    b = T.Batch(specs)
    x1 = b.read(1, T.FIELD_X)
    top = int(np.argmax(specs[1].verts[:, 2] - 1e-3 * np.abs(specs[1].verts[:, 0])))
    assert specs[1].dirichlet[top] == 0
    x1[top, 2] += 1e3
    b.write(1, T.FIELD_X, x1)
    rc, per, st = b.step(0)
    assert per[1] == T.NAN, T.STATUS_NAMES[per[1]]
    assert per[0] == T.OK
    assert np.array_equal(b.read(1, T.FIELD_X), x1)  # rolled back
    alone = T.Scene(specs[0])
    r, _ = alone.step(0)
    assert r == T.OK
    assert np.array_equal(b.read(0, T.FIELD_X), alone.read(T.FIELD_X))
    alone.close()
    b.close()
