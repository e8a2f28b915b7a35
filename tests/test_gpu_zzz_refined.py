"""FP64 with FP32 PCG passes and FP64 residual refinement (TACCEL_FP64_REFINED): the Newton
system is formed in FP64 as in FP64 mode; the PCG iterations run on its FP32 copy, and the FP64
residual decides whether another pass solves for a correction.  The converged state must meet
the FP64 bar: max |x_gpu - x_oracle| <= 1e-8 * L (L the rest bounding-box diagonal) on
teacher-forced steps, at the default PCG tolerance and at one (1e-7) that a single FP32 pass
cannot meet, so that refinement passes run.  A batch equals its scenes run alone, bit for bit.
Collected last: a new mode, after the established files.
"""
import numpy as np
import pytest

from paper_2504_12908_amd import scenes as S

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def T():
    from paper_2504_12908_amd import taccel
    taccel.lib()
    return taccel


@pytest.mark.parametrize("eta", [0.0, 1e-7])
def test_refined_cube_teacher_forced(T, oracle_lib, eta):
    spec = S.pad_press_cube(0)
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec, precision=T.FP64_REFINED, pcg_eta=eta)
    L = o.scale
    T.profile_reset()
    T.profile_enable(True)
    try:
        for k in range(4):
            g.set_state(*o.get_state())
            rc_o, st_o = o.step(k)
            rc_g, st_g = g.step(k)
            assert rc_o == 0 and rc_g == T.OK, (k, rc_o, T.STATUS_NAMES[rc_g], st_g)
            err = np.abs(g.get_state()[0] - o.get_state()[0]).max()
            say(f"  eta {eta} step {k}: newton {st_g['newton_iters']}/{st_o['newton_iters']} "
                f"pcg {st_g['pcg_iters']} err {err:.3e} (tol {1e-8 * L:.3e})")
            assert err <= 1e-8 * L
    finally:
        T.profile_enable(False)
    ref = T.profile_query("refine")
    say(f"  FP32 passes {ref['launches']} for {int(ref['bytes'])} Newton directions")
    assert ref["launches"] >= ref["bytes"] > 0
    if eta == 1e-7:
        assert ref["launches"] > ref["bytes"], ref
    g.close()


def test_refined_benchmark_scene_teacher_forced(T, oracle_lib):
    spec = S.pad_press_slide_hull(0)
    say(f"refined full-size teacher-forced steps: {spec.name}")
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec, precision=T.FP64_REFINED)
    L = o.scale
    for k in range(2):
        g.set_state(*o.get_state())
        rc_o, st_o = o.step(k)
        rc_g, st_g = g.step(k)
        assert rc_o == 0 and rc_g == T.OK, (k, rc_o, T.STATUS_NAMES[rc_g], st_g)
        xo, _, qo, _ = o.get_state()
        xg, _, qg, _ = g.get_state()
        err = max(np.abs(xg - xo).max(), np.abs(qg[:, :3] - qo[:, :3]).max())
        say(f"  step {k}: newton {st_g['newton_iters']}/{st_o['newton_iters']} pcg {st_g['pcg_iters']} "
            f"err {err:.3e} (tol {1e-8 * L:.3e})")
        assert err <= 1e-8 * L
    g.close()


def test_refined_batch_equals_single(T):
    specs = [S.batch_member(i) for i in (0, 5, 9)]
    b = T.Batch(specs, precision=T.FP64_REFINED)
    alone = [T.Scene(sp, precision=T.FP64_REFINED) for sp in specs]
    for k in range(3):
        rc, per, _ = b.step(k)
        assert rc == T.OK and list(per) == [0, 0, 0], per
        for i, sc in enumerate(alone):
            assert sc.step(k)[0] == T.OK
            assert np.array_equal(sc.read(T.FIELD_X), b.read(i, T.FIELD_X)), (k, i)
            assert np.array_equal(sc.read(T.FIELD_Q), b.read(i, T.FIELD_Q)), (k, i)
    for sc in alone:
        sc.close()
    b.close()
