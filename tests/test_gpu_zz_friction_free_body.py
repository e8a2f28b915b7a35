"""GPU parity of a free body with friction: a cube resting on the pad, launched sideways,
teacher-forced against the oracle (settling and sliding steps within 1e-8 * L)."""
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


def test_friction_sliding_cube_teacher_forced(T, oracle_lib):
    """A free cube resting on the pad with friction, launched sideways: teacher-forced
    settling and sliding steps within 1e-8 * L of the oracle."""
    spec = S.cube_resting_on_pad(0.1)
    say(f"teacher-forced steps: {spec.name} (free body, friction)")
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec)
    L = o.scale
    steps = [0, 1, 2] + list(range(3, 12)) + [12, 13, 14]
    for k in steps:
        if k == 12:
            x, v, q, qd = o.get_state()
            qd[0, 0] = 0.05
            o.set_state(x, v, q, qd)
        x, v, q, qd = o.get_state()
        if k in (3, 4, 5, 6, 7, 8, 9, 10, 11):  # settling: oracle only
            assert o.step(k)[0] == 0
            continue
        g.set_state(x, v, q, qd)
        rc_o, _ = o.step(k)
        rc_g, st_g = g.step(k)
        assert rc_o == 0 and rc_g == T.OK, (k, T.STATUS_NAMES[rc_g], st_g)
        xo, _, qo, qdo = o.get_state()
        xg, _, qg, qdg = g.get_state()
        err = max(np.abs(xg - xo).max(), np.abs(qg[:, :3] - qo[:, :3]).max())
        say(f"  step {k}: newton {st_g['newton_iters']} vx gpu {qdg[0, 0]:.6e} oracle {qdo[0, 0]:.6e} "
            f"err {err:.3e} (tol {1e-8 * L:.3e})")
        assert err <= 1e-8 * L
