"""GPU parity: the HIP path (through the C-ABI) against the CPU FP64 oracle.

Element level (neo-Hookean tets, barrier pairs, CCD, ARAP): same inputs on both sides,
relative tolerances from FP64 rounding of the two independent derivations.  Candidate sets:
bit-exact.  Whole time steps: teacher-forced (both sides start from the oracle's state),
max |x_gpu - x_oracle| <= 1e-8 * L with L the rest bounding-box diagonal of the scene.
"""
import numpy as np
import pytest

from paper_2504_12908_amd import scenes as S

pytestmark = pytest.mark.gpu

DHAT = 1e-4
MU = S.GEL_E / (2 * (1 + S.GEL_NU))
LAM = S.GEL_E * S.GEL_NU / ((1 + S.GEL_NU) * (1 - 2 * S.GEL_NU))


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def T():
    from paper_2504_12908_amd import taccel
    taccel.lib()
    return taccel


def _rand_rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def test_fem_parity(T, oracle_lib):
    say("fem parity: 64 tets")
    rng = np.random.default_rng(101)
    rest, x = [], []
    for k in range(64):
        r = np.array([[0, 0, 0], [1e-3, 0, 0], [0, 1e-3, 0], [0, 0, 1e-3]]) + rng.uniform(-2e-4, 2e-4, (4, 3))
        F = np.eye(3) if k == 0 else (np.eye(3) * 0.7 if k == 1 else
                                      _rand_rot(rng) @ (np.eye(3) + rng.uniform(-0.3, 0.3, (3, 3))))
        if np.linalg.det(F) <= 0:
            F = np.eye(3)
        rest.append(r)
        x.append(r @ F.T + rng.uniform(-1e-6, 1e-6, (4, 3)))
    rest, x = np.array(rest), np.array(x)
    e, g, H, Hp = T.debug_fem(rest, x, S.GEL_E, S.GEL_NU)
    for k in range(64):
        eo, go, Ho, Hpo = oracle_lib.nh_tet(rest[k], x[k], MU, LAM)
        sc = np.abs(Ho).max()
        assert abs(e[k] - eo) <= 1e-12 * sc * 1e-6 + 1e-12 * abs(eo)
        assert np.abs(g[k] - go).max() <= 1e-12 * sc * 1e-3
        assert np.abs(H[k] - Ho).max() <= 1e-11 * sc
        assert np.abs(Hp[k] - Hpo).max() <= 1e-11 * sc


def _pair_configs(rng, n):
    out = []
    for k in range(n):
        kind = k % 2
        if kind == 0:
            tri = rng.uniform(-1e-3, 1e-3, (3, 3))
            nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
            nrm /= np.linalg.norm(nrm)
            p = tri[0] + rng.uniform(-0.3, 1.3) * (tri[1] - tri[0]) * rng.uniform(0, 1) + \
                rng.uniform(-0.3, 1.0) * (tri[2] - tri[0]) * rng.uniform(0, 1) + nrm * rng.uniform(1e-5, 9e-5)
            x = np.concatenate([p, tri.ravel()])
            meps = 0.0
        else:
            a0, a1 = rng.uniform(-1e-3, 1e-3, 3), rng.uniform(-1e-3, 1e-3, 3)
            q = a0 + rng.uniform(-0.2, 1.2) * (a1 - a0)
            dn = np.cross(a1 - a0, rng.standard_normal(3))
            dn /= np.linalg.norm(dn)
            b0 = q + dn * rng.uniform(1e-5, 9e-5)
            v = rng.standard_normal(3) if k % 8 != 1 else (a1 - a0) + 1e-3 * rng.standard_normal(3) * np.linalg.norm(a1 - a0)
            b1 = b0 + v / np.linalg.norm(v) * 1e-3 * rng.uniform(0.5, 1.5)
            x = np.concatenate([a0, a1, b0, b1])
            meps = 1e-3 * np.sum((a1 - a0) ** 2) * np.sum((b1 - b0) ** 2)
        out.append((kind, x, meps))
    return out


def test_barrier_parity(T, oracle_lib):
    say("barrier parity: 256 pairs")
    rng = np.random.default_rng(202)
    cfg = _pair_configs(rng, 256)
    kinds = np.array([c[0] for c in cfg])
    X = np.array([c[1] for c in cfg])
    M = np.array([c[2] for c in cfg])
    e, g, H, Hp, t = T.debug_barrier(kinds, X, M, DHAT, 1e3)
    nact = 0
    for k in range(len(cfg)):
        eo, go, Ho, Hpo, to = oracle_lib.pair_barrier(kinds[k], X[k], M[k], DHAT, 1e3)
        if eo == 0.0:
            assert e[k] == 0.0
            continue
        nact += 1
        sc = np.abs(Ho).max()
        # b(d) amplifies rounding of d near dhat: relative 1e-9 plus an absolute floor at
        # 1e-12 of the barrier scale kappa * dhat^2
        assert abs(e[k] - eo) <= 1e-9 * abs(eo) + 1e-12 * 1e3 * DHAT ** 2
        assert np.abs(g[k] - go).max() <= 1e-9 * np.abs(go).max()
        assert np.abs(H[k] - Ho).max() <= 1e-7 * sc
        assert np.abs(Hp[k] - Hpo).max() <= 1e-7 * sc
    assert nact > 100


def test_friction_parity(T, oracle_lib):
    """Friction potential of 256 pairs (lagged at xn, evaluated at x = xn + a displacement in
    the static or the sliding regime): lambda, energy, gradient and Hessian of the HIP path
    against the oracle's jets."""
    say("friction parity: 256 pairs")
    rng = np.random.default_rng(303)
    cfg = _pair_configs(rng, 256)
    kinds = np.array([c[0] for c in cfg])
    XN = np.array([c[1] for c in cfg])
    M = np.array([c[2] for c in cfg])
    eh, mu = 1e-5, 0.5
    scale = np.where(np.arange(256) % 4 < 2, 0.3 * eh, 5 * eh)
    X = XN + rng.standard_normal(XN.shape) * scale[:, None] / 2
    lam, e, g, H = T.debug_friction(kinds, XN, X, M, DHAT, 1e3, mu, eh)
    nact = 0
    for k in range(len(cfg)):
        lo, eo, go, Ho = oracle_lib.pair_friction(kinds[k], XN[k], X[k], M[k], DHAT, 1e3, mu, eh)
        if lo == 0.0:
            assert lam[k] == 0.0 and e[k] == 0.0
            continue
        nact += 1
        assert abs(lam[k] - lo) <= 1e-10 * lo
        assert abs(e[k] - eo) <= 1e-9 * abs(eo)
        assert np.abs(g[k] - go).max() <= 1e-8 * np.abs(go).max()
        assert np.abs(H[k] - Ho).max() <= 1e-7 * np.abs(Ho).max()
    assert nact > 200


def test_ccd_parity(T, oracle_lib):
    say("ccd parity: 512 pairs")
    rng = np.random.default_rng(303)
    n = 512
    kinds = np.arange(n) % 2
    X = rng.uniform(-1e-3, 1e-3, (n, 12))
    P = rng.uniform(-2e-3, 2e-3, (n, 12))
    t = T.debug_ccd(kinds, X, P)
    ref = np.array([oracle_lib.accd(kinds[k], X[k], P[k]) for k in range(n)])
    assert np.abs(t - ref).max() <= 1e-12
    assert (t < 1).sum() > 20


def test_arap_parity(T, oracle_lib):
    say("arap parity: 32 matrices")
    rng = np.random.default_rng(404)
    A = np.array([_rand_rot(rng) @ (np.eye(3) + rng.uniform(-0.2, 0.2, (3, 3))) for _ in range(32)])
    e, g, H, Hp = T.debug_arap(A)
    for k in range(32):
        eo, go, Ho, Hpo = oracle_lib.arap(A[k])
        assert abs(e[k] - eo) <= 1e-12 * abs(eo) + 1e-30
        assert np.abs(g[k] - go).max() <= 1e-12 * np.abs(go).max()
        assert np.abs(H[k] - Ho).max() <= 1e-11 * np.abs(Ho).max()
        assert np.abs(Hp[k] - Hpo).max() <= 1e-11 * np.abs(Ho).max()


def _canon(rows):
    return sorted(tuple(int(v) for v in r) for r in rows)


@pytest.mark.parametrize("which", ["cube", "hull"])
def test_candidates_bit_exact(T, oracle_lib, which):
    spec = S.pad_press_cube(4) if which == "cube" else S.pad_press_slide_hull(1)
    say(f"candidates bit-exact: {spec.name}")
    g = T.Scene(spec)
    o = oracle_lib.OracleScene(spec)
    rng = np.random.default_rng(505)
    P0 = o.world_positions()
    nv = spec.verts.shape[0]
    P0[nv:, 2] -= 0.05e-3 - 3e-5   # body within dhat of the pad
    for trial in range(3):
        Pa = P0 + rng.uniform(-3e-5, 3e-5, P0.shape) * (trial > 0)
        Pb = Pa + rng.uniform(-3e-4, 3e-4, P0.shape)
        for P1 in (None, Pb):
            got = _canon(g.candidates(Pa, P1))
            ref = _canon(o.candidates(Pa, P1))
            say(f"  trial {trial} swept={P1 is not None}: gpu {len(got)} oracle {len(ref)}")
            assert got == ref
            assert len(ref) > 0
    g.close()


@pytest.mark.parametrize("seed", [0, 3])
def test_c1_step_teacher_forced(T, oracle_lib, seed):
    spec = S.pad_press_cube(seed)
    say(f"teacher-forced steps: {spec.name}")
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec)
    L = o.scale
    worst = 0.0
    for k in range(spec.n_steps):
        x, v, q, qd = o.get_state()
        g.set_state(x, v, q, qd)
        rc_o, st_o = o.step(k)
        rc_g, st_g = g.step(k)
        assert rc_o == 0 and rc_g == T.OK, (k, rc_o, T.STATUS_NAMES[rc_g], st_g)
        xo, vo, qo, qdo = o.get_state()
        xg, vg, qg, qdg = g.get_state()
        err = max(np.abs(xg - xo).max(), np.abs(qg[:, :3] - qo[:, :3]).max())
        worst = max(worst, err)
        say(f"  step {k}: newton gpu {st_g['newton_iters']} oracle {st_o['newton_iters']} "
            f"al {st_g['al_rounds']}/{st_o['al_rounds']} pcg {st_g['pcg_iters']} "
            f"active {st_g['n_active']} err {err:.3e} (tol {1e-8 * L:.3e})")
        assert err <= 1e-8 * L
    g.close()


def test_moving_dirichlet_teacher_forced(T, oracle_lib):
    """Moving Dirichlet vertices (flag 2, bottom face raised 0.04 mm per step into a held
    cube): teacher-forced steps within 1e-8 * L of the oracle, moving vertices exact."""
    spec = S.pad_push_moving(0, n_steps=6)
    say(f"teacher-forced steps: {spec.name}")
    mov = np.flatnonzero(spec.dirichlet == 2)
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec)
    L = o.scale
    for k in range(spec.n_steps):
        x, v, q, qd = o.get_state()
        g.set_state(x, v, q, qd)
        rc_o, st_o = o.step(k)
        rc_g, st_g = g.step(k)
        assert rc_o == 0 and rc_g == T.OK, (k, rc_o, T.STATUS_NAMES[rc_g], st_g)
        xo = o.get_state()[0]
        xg = g.get_state()[0]
        assert np.array_equal(xg[mov], spec.dirichlet_targets[k])
        err = np.abs(xg - xo).max()
        say(f"  step {k}: newton gpu {st_g['newton_iters']} oracle {st_o['newton_iters']} "
            f"active {st_g['n_active']} err {err:.3e} (tol {1e-8 * L:.3e})")
        assert err <= 1e-8 * L
    g.close()


def test_friction_step_teacher_forced(T, oracle_lib):
    """Friction (mu = 0.5): a cube pressed into the pad and slid; teacher-forced steps
    within 1e-8 * L of the oracle."""
    spec = S.pad_press_slide_friction(0, n_steps=6)
    say(f"teacher-forced steps: {spec.name}")
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec)
    L = o.scale
    for k in range(spec.n_steps):
        x, v, q, qd = o.get_state()
        g.set_state(x, v, q, qd)
        rc_o, st_o = o.step(k)
        rc_g, st_g = g.step(k)
        assert rc_o == 0 and rc_g == T.OK, (k, rc_o, T.STATUS_NAMES[rc_g], st_g)
        xo, _, qo, _ = o.get_state()
        xg, _, qg, _ = g.get_state()
        err = max(np.abs(xg - xo).max(), np.abs(qg[:, :3] - qo[:, :3]).max())
        say(f"  step {k}: newton gpu {st_g['newton_iters']} oracle {st_o['newton_iters']} "
            f"al {st_g['al_rounds']}/{st_o['al_rounds']} err {err:.3e} (tol {1e-8 * L:.3e})")
        assert err <= 1e-8 * L
    g.close()


def test_friction_batch_equals_single(T):
    """Friction and frictionless scenes in one batch: each scene bit for bit equal to the
    same scene run alone."""
    specs = [S.pad_press_slide_friction(0, n_steps=6), S.batch_member(0),
             S.pad_press_slide_friction(2, n_steps=6, mu=0.3)]
    say("friction batch of 3 vs single scenes, 4 steps")
    b = T.Batch(specs)
    singles = [T.Scene(s) for s in specs]
    for k in range(4):
        rc, per, st = b.step(k)
        assert rc == T.OK, per
        for i, sg in enumerate(singles):
            r, _ = sg.step(k)
            assert r == T.OK
            assert np.array_equal(b.read(i, T.FIELD_X), sg.read(T.FIELD_X))
    b.close()
    for sg in singles:
        sg.close()


@pytest.mark.parametrize("seed", [1, 2, 5])
def test_c1_mixed_precision_teacher_forced(T, oracle_lib, seed):
    """Mixed precision (FP32 Hessian/SpMV/PCG, FP64 gradient, contact and CCD): every
    teacher-forced step within 1e-4 of the pad thickness (4 mm) of the FP64 oracle."""
    spec = S.pad_press_cube(seed)
    say(f"mixed precision teacher-forced steps: {spec.name}")
    o = oracle_lib.OracleScene(spec)
    g = T.Scene(spec, precision=T.MIXED)
    tol = 1e-4 * 4e-3
    for k in range(spec.n_steps):
        x, v, q, qd = o.get_state()
        g.set_state(x, v, q, qd)
        rc_o, _ = o.step(k)
        rc_g, st_g = g.step(k)
        assert rc_o == 0 and rc_g == T.OK, (k, T.STATUS_NAMES[rc_g], st_g)
        err = np.abs(g.read(T.FIELD_X) - o.get_state()[0]).max()
        say(f"  step {k}: newton {st_g['newton_iters']} pcg {st_g['pcg_iters']} err {err:.3e} (tol {tol:.1e})")
        assert err <= tol
    g.close()


def test_batch_equals_single(T):
    specs = [S.batch_member(i) for i in range(3)]
    say("batch of 3 vs single scenes, 2 steps")
    b = T.Batch(specs)
    singles = [T.Scene(s) for s in specs]
    for k in range(2):
        rc, per, st = b.step(k)
        assert rc == T.OK, per
        for i, sg in enumerate(singles):
            r, _ = sg.step(k)
            assert r == T.OK
            assert np.array_equal(b.read(i, T.FIELD_X), sg.read(T.FIELD_X))
    b.close()
    for sg in singles:
        sg.close()
