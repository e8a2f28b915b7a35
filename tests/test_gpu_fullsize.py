"""Parity at the benchmark sizes, in the configurations bench.py times.

* The benchmark scene itself (5,775-vertex pad, 796-triangle hull, FP64, one scene): three
  teacher-forced steps of the press (both sides start every step from the oracle's state),
  max |x_gpu - x_oracle| <= 1e-8 * L, L the rest bounding-box diagonal (the slide phase is in
  test_gpu_zy_slide_phase.py, collected late: it runs 75 steps).
* The 256-scene uniform batch is in test_gpu_zzzz_batch256.py, collected last.
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


def test_benchmark_scene_teacher_forced(T, oracle_lib):
    spec = S.pad_press_slide_hull(0)
    say(f"full-size teacher-forced steps: {spec.name} ({spec.verts.shape[0]} verts)")
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec)
    L = o.scale
    for k in range(3):
        x, v, q, qd = o.get_state()
        g.set_state(x, v, q, qd)
        rc_o, st_o = o.step(k)
        rc_g, st_g = g.step(k)
        assert rc_o == 0 and rc_g == T.OK, (k, rc_o, T.STATUS_NAMES[rc_g], st_g)
        xo, _, qo, _ = o.get_state()
        xg, _, qg, _ = g.get_state()
        err = max(np.abs(xg - xo).max(), np.abs(qg[:, :3] - qo[:, :3]).max())
        say(f"  step {k}: newton gpu {st_g['newton_iters']} oracle {st_o['newton_iters']} "
            f"active {st_g['n_active']} err {err:.3e} (tol {1e-8 * L:.3e})")
        assert err <= 1e-8 * L
    g.close()
