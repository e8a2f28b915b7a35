"""The rest of the C-ABI boundary through the library: the active-pair field (Sec. 3.2 Eq. 2:
the pairs of the barrier sum), the last step's statistics, the device-pointer readout and the
reset to the creation state (the paper's API resets environments and reads their state,
Sec. 4.3).

CONTACTS is checked bit for bit against the oracle's brute-force pairs filtered by its own
squared distance; read_device against taccel_state_read byte for byte; a reset scene repeats
its first step bit for bit.
"""
import os

import numpy as np
import pytest

from paper_2504_12908_amd import scenes as S

pytestmark = pytest.mark.gpu

HOST_BUILD = bool(os.environ.get("TACCEL_TEST_HOST_LIB"))


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def T():
    from paper_2504_12908_amd import taccel
    taccel.lib()
    return taccel


def _oracle_active(B, o, P):
    import ctypes as C
    n = B.lib().orc_candidates(o.h, P.ctypes.data_as(C.POINTER(C.c_double)), None, None, 0)
    co = np.zeros((max(n, 1), 5), dtype=np.int32)
    B.lib().orc_candidates(o.h, P.ctypes.data_as(C.POINTER(C.c_double)), None,
                           co.ctypes.data_as(C.POINTER(C.c_int32)), n)
    keep = []
    for rec in co[:n]:
        x12 = np.concatenate([P[w] for w in rec[1:]])
        if B.pair_sqdist(int(rec[0]), x12)[0] < S.DHAT ** 2:
            keep.append(tuple(int(v) for v in rec))
    return sorted(keep)


def test_contacts_field_matches_oracle(T, oracle_lib):
    B = oracle_lib
    spec = S.pad_press_cube(0)
    g = T.Scene(spec)
    o = B.OracleScene(spec)
    for k in range(4):
        assert g.step(k)[0] == T.OK
    # the oracle's positions come from the GPU state, so both sides see the same point
    x, v, q, qd = g.get_state()
    o.set_state(x, v, q, qd)
    P = o.world_positions()
    ref = _oracle_active(B, o, P)
    got = sorted(map(tuple, g.contacts().tolist()))
    say(f"contacts after 4 steps: {len(got)} pairs (oracle {len(ref)})")
    assert len(ref) > 0
    assert got == ref
    st = g.stats()
    assert st["status"] == T.OK and st["newton_iters"] > 0
    g.close()


def _device_buffer(nbytes):
    """Device memory of nbytes: a torch CUDA tensor on the GPU; host memory on the host build,
    whose 'device' memory is host memory."""
    if HOST_BUILD:
        buf = np.zeros(nbytes // 8)
        return buf, buf.ctypes.data, lambda: buf.copy()
    import torch
    t = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0")
    return t, t.data_ptr(), lambda: t.cpu().numpy()


@pytest.mark.parametrize("field", ["X", "V", "Q", "QDOT", "BODY_X"])
def test_read_device_equals_read(T, field):
    f = getattr(T, "FIELD_" + field)
    spec = S.pad_press_cube(1)
    g = T.Scene(spec)
    for k in range(2):
        assert g.step(k)[0] == T.OK
    host = g.read(f)
    keep, ptr, fetch = _device_buffer(host.nbytes)
    g.read_device(f, ptr, host.nbytes)
    dev = fetch().reshape(host.shape)
    assert np.array_equal(dev, host), np.abs(dev - host).max()
    with pytest.raises(T.TaccelError):
        g.read_device(f, ptr, host.nbytes - 8)
    g.close()


def test_reset_repeats_first_steps(T):
    spec = S.pad_press_cube(2)
    g = T.Scene(spec)
    first = []
    for k in range(2):
        assert g.step(k)[0] == T.OK
        first.append(g.get_state())
    g.reset()
    assert g.stats()["newton_iters"] == 0
    x0 = g.read(T.FIELD_X)
    assert np.array_equal(x0, spec.verts)
    for k in range(2):
        assert g.step(k)[0] == T.OK
        for a, b in zip(first[k], g.get_state()):
            assert np.array_equal(a, b)
    g.close()


def test_batch_reset_mask(T):
    specs = [S.batch_member(i) for i in range(3)]
    b = T.Batch(specs)
    rc, per, st = b.step(0)
    assert rc == T.OK
    moved = [b.read(i, T.FIELD_Q) for i in range(3)]
    b.reset(np.array([1, 0, 1]))
    for i in range(3):
        q = b.read(i, T.FIELD_Q)
        if i == 1:
            assert np.array_equal(q, moved[1])
            assert b.stats(1)["newton_iters"] > 0
        else:
            assert np.array_equal(b.read(i, T.FIELD_X), specs[i].verts)
            assert np.array_equal(b.read(i, T.FIELD_V), np.zeros_like(specs[i].verts))
            assert b.stats(i)["newton_iters"] == 0
    b.close()


def _oracle_system_in_caller_nodes(o, nv, nb):
    e, G, blocks, node_of = o.system()
    to_ext = {}
    for i in range(nv):
        if node_of[i] >= 0:
            to_ext[int(node_of[i])] = i
    for b in range(nb):
        if node_of[nv + b] >= 0:
            for j in range(4):
                to_ext[int(node_of[nv + b]) + j] = nv + 4 * b + j
    g = np.zeros((nv + 4 * nb, 3))
    for n, ext in to_ext.items():
        g[ext] = G[n]
    H = {(to_ext[r], to_ext[c]): v for (r, c), v in blocks.items()}
    return g, H


@pytest.mark.parametrize("case", ["cube_step0", "cube_step6_teacher_forced", "friction_step2"])
def test_newton_system_matches_oracle(T, oracle_lib, case):
    """The assembled Newton system (gradient and every 3x3 block of the projected Hessian) of
    the first iteration of a step, GPU against the oracle's plain assembly: the same block
    pattern, and every entry within 1e-12 of the largest (measured: about 2e-15)."""
    B = oracle_lib
    if case.startswith("friction"):
        spec = S.pad_press_slide_friction(0, n_steps=6)
    else:
        spec = S.pad_press_cube(0)
    k = {"cube_step0": 0, "cube_step6_teacher_forced": 6, "friction_step2": 2}[case]
    g = T.Scene(spec)
    o = B.OracleScene(spec)
    for j in range(k):
        assert o.step(j)[0] == 0
    if k:
        g.set_state(*o.get_state())  # also clears the GPU's carried multipliers
    grad, H = g.debug_system(k)
    assert o.step_begin(k) == 0
    nv, nb = len(spec.verts), len(spec.bodies)
    go, Ho = _oracle_system_in_caller_nodes(o, nv, nb)
    gs = np.abs(go).max()
    hs = max(np.abs(v).max() for v in Ho.values())
    say(f"{case}: {len(H)} blocks (oracle {len(Ho)}), |G| {gs:.3e}, |H| {hs:.3e}")
    assert set(H) == set(Ho)
    assert np.abs(grad - go).max() <= 1e-12 * gs
    err = max(np.abs(H[key] - Ho[key]).max() for key in Ho)
    say(f"  max |dG| {np.abs(grad - go).max():.3e}, max |dH| {err:.3e}")
    assert err <= 1e-12 * hs
    # the call leaves the state where it was: the step itself still matches the oracle's
    rc, st = g.step(k)
    assert rc == T.OK and o.step_finish()[0] == 0
    assert np.abs(g.read(T.FIELD_X) - o.get_state()[0]).max() <= 1e-8 * o.scale
    g.close()
