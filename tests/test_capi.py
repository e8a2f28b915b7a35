"""C-ABI boundary checks that need no GPU: the library loads and exports every function
that include/taccel.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "taccel.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(taccel_[a-z_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = _declared()
    for required in ("taccel_scene_create", "taccel_step", "taccel_state_read",
                     "taccel_state_write", "taccel_scene_destroy", "taccel_batch_create",
                     "taccel_batch_step", "taccel_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2504_12908_amd import taccel
    if not os.path.exists(taccel.LIB_PATH):
        pytest.skip("libtaccel.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(taccel.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.taccel_status_str.restype = ctypes.c_char_p
    assert lib.taccel_status_str(0) == b"OK"
    assert lib.taccel_status_str(4) == b"LINESEARCH_FAILED"


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_2504_12908_amd import taccel
    monkeypatch.setattr(taccel, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(taccel, "_lib", None)
    with pytest.raises(RuntimeError):
        taccel.lib()


# ---------------------------------------------------------------- argument validation
# The library validates a scene description on the host before any device call, so these
# error paths run without a GPU.
def _lib_or_skip():
    from paper_2504_12908_amd import taccel
    if not os.path.exists(taccel.LIB_PATH):
        pytest.skip("libtaccel.so not built")
    return taccel


def _bad_spec(mutate):
    import copy

    from paper_2504_12908_amd import scenes
    spec = copy.deepcopy(scenes.pad_press_cube(0))
    mutate(spec)
    return spec


def _expect_arg_error(T, spec, needle):
    with pytest.raises(T.TaccelError) as ei:
        T.Scene(spec)
    assert ei.value.status == T.ERR_ARG
    assert needle in str(ei.value)


def test_rejects_inverted_tet():
    T = _lib_or_skip()

    def m(s):
        s.tets[5, 1], s.tets[5, 2] = s.tets[5, 2], s.tets[5, 1]
    _expect_arg_error(T, _bad_spec(m), "inverted or degenerate tet 5")


def test_rejects_tet_index_out_of_range():
    T = _lib_or_skip()

    def m(s):
        s.tets[0, 0] = len(s.verts)
    _expect_arg_error(T, _bad_spec(m), "tet index out of range")


def test_rejects_bad_dirichlet_flag():
    T = _lib_or_skip()

    def m(s):
        s.dirichlet[3] = 7
    _expect_arg_error(T, _bad_spec(m), "dirichlet flag")


def test_rejects_inside_out_body():
    T = _lib_or_skip()

    def m(s):
        s.bodies[0].tris = s.bodies[0].tris[:, ::-1].copy()
    _expect_arg_error(T, _bad_spec(m), "no positive volume")


def test_rejects_nonpositive_time_step():
    T = _lib_or_skip()

    def m(s):
        s.params["h"] = 0.0
    _expect_arg_error(T, _bad_spec(m), "must be > 0")


def test_rejects_body_triangle_index():
    T = _lib_or_skip()

    def m(s):
        s.bodies[0].tris[2, 1] = 99
    _expect_arg_error(T, _bad_spec(m), "body triangle index out of range")


# ---------------------------------------------------------------- serving, host side only
def test_server_rejects_bad_params():
    T = _lib_or_skip()
    with pytest.raises(T.TaccelError) as ei:
        T.Server(hbm_budget_bytes=0.0)
    assert ei.value.status == T.ERR_ARG


def test_server_submit_validates_on_host():
    # the scene is checked before it is queued: nothing reaches the device
    T = _lib_or_skip()
    srv = T.Server(hbm_budget_bytes=1e9)

    def m(s):
        s.tets[5, 1], s.tets[5, 2] = s.tets[5, 2], s.tets[5, 1]
    with pytest.raises(T.TaccelError) as ei:
        srv.submit(_bad_spec(m), 3)
    assert ei.value.status == T.ERR_ARG
    assert "inverted or degenerate tet 5" in str(ei.value)
    assert srv.info()["queued"] == 0
    assert srv.poll(wait_ms=0) == []
    srv.close()


def test_mixed_batch_of_several_scenes_is_refused():
    T = _lib_or_skip()
    from paper_2504_12908_amd import scenes
    with pytest.raises(T.TaccelError) as ei:
        T.Batch([scenes.pad_press_cube(0), scenes.pad_press_cube(1)], precision=T.MIXED)
    assert ei.value.status == T.ERR_ARG
    assert "one scene per batch" in str(ei.value)


def test_rejects_bad_precision_and_forcing():
    T = _lib_or_skip()

    def m(s):
        s.params["pcg_forcing"] = 2
    _expect_arg_error(T, _bad_spec(m), "pcg_forcing must be 0 or 1")
    from paper_2504_12908_amd import scenes
    with pytest.raises(T.TaccelError) as ei:
        T.Scene(scenes.pad_press_cube(0), precision=7)
    assert ei.value.status == T.ERR_ARG
    assert "precision must be" in str(ei.value)


def test_refined_and_fp64_scenes_do_not_share_a_batch():
    T = _lib_or_skip()
    from paper_2504_12908_amd import scenes
    a = T._Desc(scenes.pad_press_cube(0), T.FP64_REFINED)
    b = T._Desc(scenes.pad_press_cube(1), T.FP64)
    ds = (T.taccel_scene_desc * 2)(a.desc, b.desc)
    out = T.C.c_void_p()
    st = T.lib().taccel_batch_create(ds, 2, None, T.C.byref(out))
    assert st == T.ERR_ARG
    assert b"same precision" in T.lib().taccel_last_error()
