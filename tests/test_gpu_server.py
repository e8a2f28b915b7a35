"""Serving path (taccel_server_*): continuous batching must not change any request's result.

Each request's final state is compared bitwise with the same scene stepped alone through
taccel_step; a request that fails stops at its failing step (rolled back) without touching
the others; budgets and cohort limits are respected.
"""
import time

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


def _alone(T, spec, n_steps, **overrides):
    sc = T.Scene(spec, **overrides)
    status = T.OK
    for k in range(n_steps):
        rc, _ = sc.step(k)
        if rc != T.OK:
            status = rc
            break
    out = sc.get_state()
    sc.close()
    return status, out


def _drain(srv, n, timeout_s=120.0):
    done = {}
    t0 = time.time()
    while len(done) < n:
        assert time.time() - t0 < timeout_s, "server did not complete the requests in time"
        for c in srv.poll(wait_ms=200):
            done[c["req_id"]] = c
    return done


def _fields(T, srv, rid):
    return [srv.read(rid, f) for f in (T.FIELD_X, T.FIELD_V, T.FIELD_Q, T.FIELD_QDOT)]


def test_server_mix_equals_alone(T):
    lengths = [3, 6, 10, 4, 8]
    specs = [S.batch_member(i) for i in range(len(lengths))]
    say("server: 5 requests of 3..10 steps plus one failing request, vs each scene alone")
    srv = T.Server(hbm_budget_bytes=8e9, max_cohort=64, max_cohorts=4, coalesce_ms=5.0)
    ids = [srv.submit(sp, n) for sp, n in zip(specs, lengths)]
    bad_spec = S.batch_member(7)
    bad = srv.submit(bad_spec, 5, max_newton=1)
    done = _drain(srv, len(ids) + 1)
    for rid, sp, n in zip(ids, specs, lengths):
        c = done[rid]
        assert c["status"] == T.OK, T.STATUS_NAMES[c["status"]]
        assert c["steps_done"] == n
        assert len(srv.step_latencies(rid)) == n
        st, ref = _alone(T, sp, n)
        assert st == T.OK
        for a, b in zip(_fields(T, srv, rid), ref):
            assert np.array_equal(a, b)
        srv.release(rid)
    c = done[bad]
    assert c["status"] == T.NOT_CONVERGED
    assert c["steps_done"] == 1
    st, ref = _alone(T, bad_spec, 5, max_newton=1)
    assert st == T.NOT_CONVERGED
    for a, b in zip(_fields(T, srv, bad), ref):
        assert np.array_equal(a, b)
    # rolled back to the initial state
    assert np.array_equal(srv.read(bad, T.FIELD_X), bad_spec.verts)
    info = srv.info()
    assert info["queued"] == 0 and info["running_cohorts"] == 0 and info["used_bytes"] == 0
    assert info["peak_bytes"] > 0
    srv.close()


def test_server_staggered_cohorts(T):
    # requests arriving while an earlier cohort runs form further, concurrent cohorts; each
    # request ends exactly as the same scene stepped alone (status, step count and state)
    specs = [S.batch_member(10 + i) for i in range(4)]
    say("server: staggered arrivals, one request per cohort, up to 4 cohorts at once")
    srv = T.Server(hbm_budget_bytes=8e9, max_cohort=1, max_cohorts=4, coalesce_ms=1.0)
    ids = []
    for sp in specs:
        ids.append(srv.submit(sp, 10))
        time.sleep(0.02)
    done = _drain(srv, len(ids))
    n_ok = 0
    for rid, sp in zip(ids, specs):
        st, ref = _alone(T, sp, 10)
        c = done[rid]
        assert c["status"] == st, (T.STATUS_NAMES[c["status"]], T.STATUS_NAMES[st])
        n_ok += c["status"] == T.OK
        for a, b in zip(_fields(T, srv, rid), ref):
            assert np.array_equal(a, b)
    assert n_ok >= 3
    assert srv.info()["running_cohorts"] == 0
    srv.close()


def test_server_refills_running_cohort(T):
    """Requests of uneven mesh sizes admitted into the slots a finished request leaves in the
    one running cohort (max_cohorts = 1): the late request finishes before the long one (it
    did not wait for the cohort to end), and every request's result is bitwise the same as
    its scene stepped alone, across the move of the long request into the rebuilt batch."""
    say("server: a late request refills a running cohort (uneven meshes)")
    short = S.batch_member(40)                                  # 243-vertex pad, 8-point hull
    long_ = S.pad_press_cube(41)                                # 243-vertex pad, cube
    late = S.pad_press_slide_hull(42, n_steps=10, cells=(4, 4, 2), n_points=10)  # 75 vertices
    srv = T.Server(hbm_budget_bytes=8e9, max_cohort=4, max_cohorts=1, coalesce_ms=1.0)
    r_short = srv.submit(short, 2)
    r_long = srv.submit(long_, 8)
    time.sleep(0.05)
    r_late = srv.submit(late, 3)
    order = []
    done = {}
    t0 = time.time()
    while len(done) < 3:
        assert time.time() - t0 < 600
        for c in srv.poll(wait_ms=50):
            done[c["req_id"]] = c
            order.append(c["req_id"])
    assert all(done[r]["status"] == T.OK for r in (r_short, r_long, r_late)), done
    assert order.index(r_late) < order.index(r_long), order
    for rid, sp, n in ((r_short, short, 2), (r_long, long_, 8), (r_late, late, 3)):
        st, ref = _alone(T, sp, n)
        assert st == T.OK
        for a, b in zip(_fields(T, srv, rid), ref):
            assert np.array_equal(a, b)
    srv.close()


def test_server_limits(T):
    say("server: one cohort at a time; a budget nothing fits")
    specs = [S.batch_member(20 + i) for i in range(3)]
    srv = T.Server(hbm_budget_bytes=8e9, max_cohort=1, max_cohorts=1)
    ids = [srv.submit(sp, 2) for sp in specs]
    seen_max = 0
    done = {}
    t0 = time.time()
    while len(done) < len(ids):
        assert time.time() - t0 < 120
        seen_max = max(seen_max, srv.info()["running_cohorts"])
        for c in srv.poll(wait_ms=20):
            done[c["req_id"]] = c
    assert seen_max <= 1
    assert all(done[r]["status"] == T.OK for r in ids)
    # the cohorts held at most their reservations, which never passed the budget
    assert 0 < srv.info()["peak_bytes"] <= 8e9
    srv.close()

    tiny = T.Server(hbm_budget_bytes=1024.0)
    rid = tiny.submit(specs[0], 2)
    c = _drain(tiny, 1)[rid]
    assert c["status"] == T.ERR_OOM and c["steps_done"] == 0
    tiny.close()


def test_server_cancel_on_destroy(T):
    say("server: destroy with queued and running requests")
    srv = T.Server(hbm_budget_bytes=8e9, max_cohort=1, max_cohorts=1)
    for i in range(3):
        srv.submit(S.batch_member(30 + i), 10)
    time.sleep(0.05)
    srv.close()  # must return: running cohort stops after its current step, the rest cancel
