"""Robot-driven scenes (Sec. 4.1: a gel pad is a tet mesh attached to a robot link by its back
face; kinematic targets from the robot's joint values) and the two-finger grasp, on the CPU
FP64 oracle, on reduced grids.

Pins fixed by mechanics rather than by the oracle itself:
* forward kinematics: every back-face vertex and every link vertex moves rigidly with its
  finger, composed from the joint values;
* a grasp that is symmetric under the half turn about the gripper axis (finger 1 is finger 0
  turned by pi, the object a centred cube) stays symmetric: the second pad is the first turned
  by pi and the object's centre stays on the axis, to the Newton tolerance;
* two pads pressed into each other (soft-soft contact) never interpenetrate;
* with Coulomb friction (App. A.3) and gravity the squeezed cube rises with the gripper, to
  5 % of the lift (measured: 0.4 %).  (Without friction it rises too: the cube sits 0.35 mm
  deep in pockets of the gel, whose walls carry its weight through normal forces.)
"""
import numpy as np
import pytest

from paper_2504_12908_amd import scenes as S

MM = S.MM
CELLS = (2, 8, 6)


def _cube_grasp(n_squeeze, n_lift, lift, friction, gravity):
    cv, ct = S.box_mesh((0, 0, 0), (8 * MM,) * 3)
    open0 = 2 * (6 * MM + 4 * MM + 0.05 * MM)
    traj = [(0.0, open0)] + [(lift * max(0, k - n_squeeze) / max(n_lift, 1),
                              open0 - 2 * (0.05 * MM + 0.3 * MM) * min(k, n_squeeze) / n_squeeze)
                             for k in range(1, n_squeeze + n_lift + 1)]
    return S.gripper_scene("cube_grasp", (cv, ct), np.array(traj), 0.005, cells=CELLS,
                           friction=friction, gravity=gravity)


def test_gripper_fk_moves_attachments_rigidly():
    spec = S.grasp_lift(0, cells=CELLS, n_points=40, n_squeeze=3, n_lift=3, lift=2 * MM)
    npv = spec.meta["pad_vertices"]
    moving = np.where(spec.dirichlet == 2)[0]
    rest = spec.verts[moving]
    traj = spec.meta["joint_traj"]
    for k in range(spec.n_steps):
        tgt = spec.dirichlet_targets[k]
        # pairwise distances within each finger's back face are those at rest
        for f in range(2):
            sel = (moving >= f * npv) & (moving < (f + 1) * npv)
            a, b = rest[sel], tgt[sel]
            da = np.linalg.norm(a[:, None] - a[None], axis=2)
            db = np.linalg.norm(b[:, None] - b[None], axis=2)
            assert np.abs(da - db).max() <= 1e-15
        # finger 0 is translated by the base joint and half the opening change
        dz = traj[k + 1][0] - traj[0][0]
        dx = -0.5 * (traj[k + 1][1] - traj[0][1])
        sel0 = moving < npv
        assert np.allclose(tgt[sel0] - rest[sel0], [dx, 0.0, dz], atol=1e-15)
        # link targets: the links move with their pads' back faces
        for f, body in enumerate(spec.bodies[1:]):
            q = spec.body_targets[k, 1 + f]
            moved = S.apply_target(body.verts, q)
            assert np.allclose(np.linalg.norm(moved[:, None] - moved[None], axis=2),
                               np.linalg.norm(body.verts[:, None] - body.verts[None], axis=2),
                               atol=1e-15)
        assert np.allclose(spec.body_targets[k, 1, 0:3], [dx, 0.0, dz], atol=1e-15)


def test_oracle_symmetric_grasp_stays_symmetric(oracle_lib):
    spec = _cube_grasp(5, 0, 0.0, 0.0, (0.0, 0.0, 0.0))
    o = oracle_lib.OracleScene(spec)
    npv = spec.meta["pad_vertices"]
    R = np.diag([-1.0, -1.0, 1.0])
    tol = 1e-8 * o.scale
    for k in range(spec.n_steps):
        rc, st = o.step(k)
        assert rc == 0, (k, st)
        x, v, q, qd = o.get_state()
        assert np.abs(x[npv:] - x[:npv] @ R.T).max() <= tol
        assert np.abs(q[0][0:2]).max() <= tol
        dmin, vmin, nact = o.diagnostics()
        assert dmin > 0.0 and vmin > 0.0 and nact > 0


def test_oracle_pad_pad_contact(oracle_lib):
    w, d = 32 * MM / CELLS[1], 24 * MM / CELLS[2]
    open0 = 2 * (6 * MM + 0.05 * MM)
    traj = [(0.0, open0)] + [(0.0, open0 - 2 * (0.05 * MM + 0.3 * MM) * min(k, 5) / 5)
                             for k in range(1, 7)]
    spec = S.gripper_scene("pad_pad", None, np.array(traj), 0.005, cells=CELLS,
                           mount1=(0.0, w / 3, d / 3))
    o = oracle_lib.OracleScene(spec)
    moving = np.where(spec.dirichlet == 2)[0]
    for k in range(spec.n_steps):
        rc, st = o.step(k)
        assert rc == 0, (k, st)
        dmin, vmin, nact = o.diagnostics()
        assert dmin > 0.0 and vmin > 0.0
        if k >= 1:
            assert nact > 100  # the coated faces are in contact
        x = o.get_state()[0]
        assert np.array_equal(x[moving], spec.dirichlet_targets[k])


def test_oracle_friction_grasp_lifts(oracle_lib):
    lift = 1.5 * MM
    spec = _cube_grasp(4, 6, lift, 0.5, (0.0, 0.0, -9.81))
    o = oracle_lib.OracleScene(spec)
    z = []
    for k in range(spec.n_steps):
        rc, st = o.step(k)
        assert rc == 0, (k, st)
        z.append(o.get_state()[2][0][2])
    assert z[3] < 0.0  # it sags under gravity while squeezed
    rise = z[-1] - z[3]
    assert abs(rise - lift) <= 0.05 * lift, rise
