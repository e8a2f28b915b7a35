"""The library's HIP sources built for the host against the emulation in ``tests/hip_host``
(every device allocation ends at a guard page and is unmapped when freed, so an access past a
buffer or after its release faults at once).  Each case runs in a fresh interpreter that loads
that build through the same C ABI; a memory error ends it with a non-zero status and the
allocation the faulting address belongs to.

Regression: a batch of 32 small pads used to fault at creation (a point query accepted an
edge entry sharing its hash bucket, and the target index was then read as a triangle's).
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def host_lib():
    sys.path.insert(0, os.path.join(HERE, "hip_host"))
    try:
        import build as hb
    finally:
        sys.path.pop(0)
    return hb.build()


PRELUDE = """
import sys
sys.path.insert(0, {root!r})
import numpy as np
from paper_2504_12908_amd import taccel as T, scenes as S
T.LIB_PATH = {lib!r}
T.lib()
from oracle import binding as B
"""


def run(lib, body, timeout=600):
    code = PRELUDE.format(root=ROOT, lib=lib) + body
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=timeout)
    assert p.returncode == 0, (p.returncode, p.stdout[-2000:], p.stderr[-4000:])
    assert "DONE" in p.stdout, p.stdout[-2000:]
    return p.stdout


def test_host_build_element_evaluators(host_lib):
    """The host build computes the same barrier and friction derivatives as the oracle."""
    run(host_lib, """
x = np.concatenate([[4e-4, 4e-4, 5e-5], [0, 0, 0, 1.5e-3, 0, 0, 0, 1.5e-3, 0]])
e, g, H, Hp, t = T.debug_barrier(np.array([0]), x[None], np.array([0.0]), 1e-4, 1e3)
eo, go, Ho, Hpo, to = B.pair_barrier(0, x, 0.0, 1e-4, 1e3)
assert abs(e[0] - eo) <= 1e-12 * abs(eo) and np.abs(Hp[0] - Hpo).max() <= 1e-9 * np.abs(Hpo).max()
xn = x.copy(); x1 = x.copy(); x1[:3] += [3e-5, -1e-5, 0.0]
lam, e, g, H = T.debug_friction(np.array([0]), xn[None], x1[None], np.array([0.0]), 1e-4, 1e3, 0.5, 1e-5)
lo, eo, go, Ho = B.pair_friction(0, xn, x1, 0.0, 1e-4, 1e3, 0.5, 1e-5)
assert abs(lam[0] - lo) <= 1e-12 * lo and abs(e[0] - eo) <= 1e-10 * abs(eo)
print("DONE")
""")


def test_host_build_candidates_match_oracle(host_lib):
    """Broad phase of one scene (pad and lowered cube) equal to the oracle's enumeration."""
    run(host_lib, """
import ctypes as C
spec = S.pad_press_cube(0)
spec.bodies[0].verts = spec.bodies[0].verts + np.array([0, 0, 5e-3])
g = T.Scene(spec)
o = B.OracleScene(spec)
P = np.zeros((o.nw, 3)); B.lib().orc_world_positions(o.h, P.ctypes.data_as(C.POINTER(C.c_double)))
P[o.nv:, 2] -= 5e-3 - 2e-5
cg = set(map(tuple, g.candidates(P)))
co = np.zeros((200000, 5), dtype=np.int32)
n = B.lib().orc_candidates(o.h, P.ctypes.data_as(C.POINTER(C.c_double)), None,
                           co.ctypes.data_as(C.POINTER(C.c_int32)), 200000)
assert cg == set(map(tuple, co[:n])) and n > 1000, (len(cg), n)
print("DONE")
""")


def test_host_build_batch_of_32_is_created(host_lib):
    """Creating a batch of 32 small pads runs the all-scene broad phase and the zero-distance
    check over its candidates; it used to fault on out-of-range targets."""
    run(host_lib, """
b = T.Batch(S.uniform_batch(32))
b.close()
print("DONE")
""")


def test_host_build_tactile_maps(host_lib):
    """Depth map and markers of the host build equal the oracle's definitions (rest state)."""
    run(host_lib, """
from oracle import tactile as TO
spec = S.pad_press_cube(0)
g = T.Scene(spec)
tris = S.top_surface_tris(spec)
idx, bary = S.marker_layout(spec, tris, 5, 5)
pos, flow = g.markers(tris[idx], bary)
po, fo = TO.markers(spec.verts, spec.verts, tris[idx], bary)
assert np.array_equal(pos, po) and np.all(flow == 0)
cam = T.camera((-11e-3, -11e-3, 0.0), (1.0, 0, 0), (0, 1.0, 0), 0.7e-3, 32, 32)
d, nrm = g.depth_map(cam, tris)
do, no = TO.depth_map(spec.verts, tris, (-11e-3, -11e-3, 0.0), (1.0, 0, 0), (0, 1.0, 0), 0.7e-3, 32, 32)
assert np.array_equal(np.isfinite(d), np.isfinite(do)) and np.array_equal(d[np.isfinite(d)], do[np.isfinite(do)])
print("DONE")
""")


def test_host_build_multiscene_newton_iterations(host_lib):
    """One Newton iteration (then the roll-back of the unconverged step) of a 32-scene batch
    and of a batch mixing friction and frictionless scenes runs without a memory error."""
    run(host_lib, """
specs = S.uniform_batch(32)
for sp in specs:
    sp.params["max_newton"] = 1
b = T.Batch(specs, pcg_eta=0.5)
rc, per, st = b.step(0)
assert set(per.tolist()) <= {0, 3}, per
b.close()
specs = [S.pad_press_slide_friction(0, n_steps=6), S.batch_member(0), S.pad_press_slide_friction(2, n_steps=6, mu=0.3)]
for sp in specs:
    sp.params["max_newton"] = 2
b = T.Batch(specs, pcg_eta=0.5)
rc, per, st = b.step(0)
assert set(per.tolist()) <= {0, 3}, per
b.close()
print("DONE")
""")


def test_host_build_fp64_refined(host_lib):
    """TACCEL_FP64_REFINED (FP32 PCG passes on an FP32 copy of the FP64 system, FP64 residual
    refinement): teacher-forced cube steps match the oracle within 1e-8 L with a PCG tolerance
    (1e-7) that one FP32 pass cannot meet, so refinement passes run (more passes than Newton
    directions; one step here, four in the GPU test file); a batch of two scenes equals each
    scene alone, bit for bit."""
    out = run(host_lib, """
spec = S.pad_press_cube(0)
o = B.OracleScene(spec)
g = T.Scene(spec, precision=T.FP64_REFINED, pcg_eta=1e-7)
T.profile_reset(); T.profile_enable(True)
for k in range(1):
    g.set_state(*o.get_state())
    rc_o, _ = o.step(k)
    rc, st = g.step(k)
    assert rc_o == 0 and rc == T.OK, (k, rc_o, rc)
    err = np.abs(g.get_state()[0] - o.get_state()[0]).max()
    assert err <= 1e-8 * o.scale, (k, err)
T.profile_enable(False)
ref = T.profile_query("refine")
print("passes", ref["launches"], "directions", ref["bytes"])
assert ref["launches"] > ref["bytes"] > 0, ref
g.close()
specs = [S.batch_member(1), S.batch_member(4)]
b = T.Batch(specs, precision=T.FP64_REFINED)
rc, per, st = b.step(0)
assert rc == T.OK and list(per) == [0, 0], per
for i, sp in enumerate(specs):
    sc = T.Scene(sp, precision=T.FP64_REFINED)
    assert sc.step(0)[0] == T.OK
    assert np.array_equal(sc.read(T.FIELD_X), b.read(i, T.FIELD_X))
    assert np.array_equal(sc.read(T.FIELD_Q), b.read(i, T.FIELD_Q))
    sc.close()
b.close()
print("DONE")
""")
    print(out)


def test_host_build_pcg_forcing(host_lib):
    """pcg_forcing = 1 (Eisenstat-Walker forcing terms for the PCG tolerance): a teacher-forced
    cube step still matches the oracle within 1e-8 L, with fewer PCG iterations than the fixed
    tolerance."""
    run(host_lib, """
spec = S.pad_press_cube(0)
o = B.OracleScene(spec)
x0 = o.get_state()
rc_o, _ = o.step(0)
assert rc_o == 0
pcg = {}
for f in (0, 1):
    g = T.Scene(spec, pcg_forcing=f)
    g.set_state(*x0)
    rc, st = g.step(0)
    assert rc == T.OK, rc
    err = np.abs(g.get_state()[0] - o.get_state()[0]).max()
    assert err <= 1e-8 * o.scale, (f, err)
    pcg[f] = st["pcg_iters"]
    g.close()
print("pcg fixed", pcg[0], "forcing", pcg[1])
assert pcg[1] < pcg[0], pcg
try:
    T.Scene(spec, pcg_forcing=2)
    raise AssertionError("pcg_forcing=2 accepted")
except T.TaccelError as e:
    assert e.status == T.ERR_ARG, e
print("DONE")
""")


def test_host_build_mixed_batch_equals_single(host_lib):
    """Mixed precision with several scenes in one batch (refused by the gfx950 build until the
    cause of its GPU fault is shown; allowed by the host build): each scene of a 3-scene mixed
    batch ends its first step bit for bit as the same scene stepped alone in mixed precision."""
    run(host_lib, """
specs = [S.batch_member(i) for i in (2, 6, 11)]
b = T.Batch(specs, precision=T.MIXED)
rc, per, st = b.step(0)
assert rc == T.OK and list(per) == [0, 0, 0], per
for i, sp in enumerate(specs):
    sc = T.Scene(sp, precision=T.MIXED)
    assert sc.step(0)[0] == T.OK
    assert np.array_equal(sc.read(T.FIELD_X), b.read(i, T.FIELD_X)), i
    assert np.array_equal(sc.read(T.FIELD_Q), b.read(i, T.FIELD_Q)), i
    sc.close()
b.close()
print("DONE")
""")


LONG = os.environ.get("TACCEL_HOST_LONG") == "1"


@pytest.mark.slow
@pytest.mark.skipif(not LONG, reason="hours of CPU: set TACCEL_HOST_LONG=1")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_host_build_256_batch_two_full_steps(host_lib, precision):
    """The 256-scene uniform batch through creation and two full steps, in FP64 and in mixed
    precision (several scenes per mixed batch are allowed in the host build only), with every
    device allocation behind guard pages: no memory error, every scene converged, every
    scene's positions finite, and (FP64) scenes 0, 97 and 255, started from the oracle's state
    each step, within 1e-8 L of the oracle.  PCG tolerance 1e-2 keeps the emulation to about
    an hour on four threads (the converged states meet the same Newton test)."""
    run(host_lib, f"""
import time
specs = S.uniform_batch(256)
fp64 = {precision == 'fp64'}
t0 = time.time()
b = T.Batch(specs, precision=T.FP64 if fp64 else T.MIXED, pcg_eta=1e-2)
print("created", time.time() - t0, flush=True)
picks = (0, 97, 255)
oracles = {{i: B.OracleScene(specs[i]) for i in picks}} if fp64 else {{}}
for k in range(2):
    for i, o in oracles.items():
        x, v, q, qd = o.get_state()
        b.write(i, T.FIELD_X, x); b.write(i, T.FIELD_V, v); b.write(i, T.FIELD_Q, q); b.write(i, T.FIELD_QDOT, qd)
    rc, per, st = b.step(k)
    print("step", k, "ok", int((per == 0).sum()), "max newton", max(s["newton_iters"] for s in st),
          time.time() - t0, flush=True)
    assert (per == 0).all(), per
    for i, o in oracles.items():
        assert o.step(k)[0] == 0
        xo, _, qo, _ = o.get_state()
        err = max(np.abs(b.read(i, T.FIELD_X) - xo).max(), np.abs(b.read(i, T.FIELD_Q)[:, :3] - qo[:, :3]).max())
        print("  scene", i, "err", err, flush=True)
        assert err <= 1e-8 * o.scale
for i in range(256):
    assert np.isfinite(b.read(i, T.FIELD_X)).all()
b.close()
print("DONE")
""", timeout=100000)
