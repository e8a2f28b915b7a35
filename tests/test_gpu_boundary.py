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
