"""Benchmark: Newton-converged env-steps/s of the IPC time step on one MI355X.

Workload (one scene, FP64): a 32x24x6 mm gel pad meshed as a 32x24x6 hex grid split into
6 tets per hex (5,775 vertices, 27,648 tets, bottom face fixed, neo-Hookean E = 0.3 MPa,
nu = 0.45) pressed by a rigid 400-point random convex hull (796 triangles, 8 mm extent)
that is lowered 1.0 mm over 50 steps and then slid 2 mm over 50 steps, h = 0.005 s,
dhat = 1e-4 m, kappa = 1e3, Newton tolerance 1e-6.  Synthetic seeded input (seed 0).

A step is one call of taccel_step (predict, Newton loops with broad phase, narrow phase,
barrier / FEM / affine-body derivatives, assembly, PCG, CCD, line search, augmented
Lagrangian rounds and snap, velocity update).  After W warm-up steps, K steps are timed
with the device synchronised on both sides.  The PCG sparse matrix-vector kernel is timed
with HIP events on the solver's stream over the timed region (roofline field).  The CPU
FP64 oracle is timed on a bounded sample of the same workload (cpu_baseline field).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Newton-converged env-steps/sec on 1 GPU; p50/p99 step latency; vs plain FP64"
HBM_PEAK_GBS = 8000.0


def cpu_baseline(spec, k_warm, k_timed):
    """Oracle on the host: warm-up steps, then time k_timed steps (one scene, one core)."""
    from oracle import binding as O

    o = O.OracleScene(spec)
    for k in range(k_warm):
        o.step(k)
    t0 = time.perf_counter()
    ok = 0
    for k in range(k_warm, k_warm + k_timed):
        rc, _ = o.step(k)
        ok += rc == 0
    dt = time.perf_counter() - t0
    return dict(value=ok / dt, unit="env-steps/s", cores=1, kind="oracle",
                sample=f"steps {k_warm}..{k_warm + k_timed - 1} of the same scene after "
                       f"{k_warm} warm-up step(s); one scene on one host core; {dt:.1f} s")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pcg_dir_spmv_pad32x24x6_hull796_fp64_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2504_12908_amd", "csrc", f) for f in ("kernels.hip", "kernels.h")]


def _kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _measured_traffic():
    """HBM bytes per launch of the sparse product from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the factor a plain device copy of
    known size gives), or None when the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != _kernel_source_hash():
        return None
    return (float(kv["fetch_kib"]) * float(kv["fetch_factor"]) +
            float(kv["write_kib"]) * float(kv["write_factor"])) * 1024.0


def _spmv_roofline(taccel):
    prof = taccel.profile_query("spmv")
    n_l = max(prof["launches"], 1)
    avg_ms = prof["total_ms"] / n_l
    bytes_per_launch = prof["bytes"] / n_l
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return dict(bound="hbm", kernel="k_pcg_dir_spmv", achieved=achieved, peak=HBM_PEAK_GBS,
                unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=None,
                launches=prof["launches"], avg_launch_us=avg_ms * 1e3,
                algorithmic_bytes_per_launch=bytes_per_launch)


def _set_friction(args, specs):
    """--friction MU: the workload with the lagged friction potential (eps_v = 1e-3 m/s)."""
    if args.friction > 0.0:
        for sp in specs:
            sp.params["friction"] = args.friction
            sp.params["eps_v"] = 1e-3


def run_single(args, taccel, scenes, np):
    spec = scenes.pad_press_slide_hull(0)
    _set_friction(args, [spec])
    W, K = args.warmup, args.steps
    if W + K > spec.n_steps:
        sys.exit(f"warmup + steps must be <= {spec.n_steps}")
    prec = taccel.MIXED if args.precision == "mixed" else taccel.FP64
    sc = taccel.Scene(spec, precision=prec)
    for k in range(W):
        rc, st = sc.step(k)
        print(f"warmup step {k}: {taccel.STATUS_NAMES[rc]} newton={st['newton_iters']} "
              f"pcg={st['pcg_iters']} {st['step_ms']:.1f} ms", file=sys.stderr, flush=True)
    taccel.device_synchronize()
    taccel.profile_reset()
    taccel.profile_enable(True)
    lat = []
    ok = 0
    stats = []
    t0 = time.perf_counter()
    for k in range(W, W + K):
        ts = time.perf_counter()
        rc, st = sc.step(k)
        lat.append((time.perf_counter() - ts) * 1e3)
        ok += rc == taccel.OK
        stats.append(st)
        if rc != taccel.OK:
            print(f"step {k} failed: {taccel.lib().taccel_last_error().decode()}", file=sys.stderr)
        print(f"step {k}: {taccel.STATUS_NAMES[rc]} newton={st['newton_iters']} "
              f"al={st['al_rounds']} pcg={st['pcg_iters']} active={st['n_active']} "
              f"{lat[-1]:.1f} ms", file=sys.stderr, flush=True)
    taccel.device_synchronize()
    dt = time.perf_counter() - t0
    taccel.profile_enable(False)
    out = dict(
        metric=METRIC, value=ok / dt, unit="env-steps/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=dt * 1e3 / K, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64" if prec == taccel.FP64 else "f32+f64", data="synthetic",
        config=dict(workload="gel pad 32x24x6 grid (5775 verts, 27648 tets) pressed and slid "
                             "by a 400-point convex hull (796 tris), 1 scene",
                    scenes=1, h=spec.params["h"], step_range=[W, W + K - 1],
                    precision=args.precision, friction=args.friction),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        newton_iters_per_step=float(np.mean([s["newton_iters"] for s in stats])),
        pcg_iters_per_step=float(np.mean([s["pcg_iters"] for s in stats])),
        roofline=_spmv_roofline(taccel),
    )
    if prec == taccel.FP64:
        out["roofline"]["traffic"] = _measured_traffic()
    pcg = taccel.profile_query("pcg")
    if pcg["launches"]:
        out["pcg_us_per_iter"] = pcg["total_ms"] * 1e3 / pcg["launches"]
    if args.phases > 0 and W + K + args.phases <= spec.n_steps:
        # after the timed region: host wall time per Newton-iteration phase (every phase ends
        # with a synchronisation here, so the sum exceeds an unprofiled iteration)
        taccel.profile_reset()
        taccel.profile_enable(False, phases=True)
        for k in range(W + K, W + K + args.phases):
            sc.step(k)
        taccel.profile_enable(False)
        ph = {name: taccel.profile_query(name) for name in taccel.PHASES}
        n_it = max(ph["solve"]["launches"], 1)
        out["phase_ms_per_newton_iter"] = {name: v["total_ms"] / n_it for name, v in ph.items()}
    sc.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, 1, 1)
        v = out["cpu_baseline"]["value"]
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / v if v > 0 else None
    return out


def run_batch(args, taccel, scenes, np):
    """Uniform batch: n copies of the small pad with seeded hull indenters, one launch per
    stage over all scenes."""
    n = args.scenes
    if n > 64:
        sys.exit("bench.py: batches of more than 64 scenes are off: a 256-scene batch once ended "
                 "in a GPU memory fault whose cause is not found yet")
    specs = scenes.uniform_batch(n)
    _set_friction(args, specs)
    W, K = args.warmup, args.steps
    if W + K > specs[0].n_steps:
        sys.exit(f"warmup + steps must be <= {specs[0].n_steps}")
    prec = taccel.MIXED if args.precision == "mixed" else taccel.FP64
    if prec == taccel.MIXED and n > 1:
        sys.exit("bench.py: mixed precision runs one scene per batch (see include/taccel.h)")
    b = taccel.Batch(specs, precision=prec)
    for k in range(W):
        rc, per, st = b.step(k)
        print(f"warmup step {k}: rc={taccel.STATUS_NAMES[rc]} {st[0]['step_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    taccel.device_synchronize()
    taccel.profile_reset()
    taccel.profile_enable(True)
    lat, ok, newton = [], 0, []
    t0 = time.perf_counter()
    for k in range(W, W + K):
        ts = time.perf_counter()
        rc, per, st = b.step(k)
        lat.append((time.perf_counter() - ts) * 1e3)
        ok += int((per == taccel.OK).sum())
        newton.append(max(s["newton_iters"] for s in st))
        print(f"step {k}: ok={int((per == taccel.OK).sum())}/{n} max_newton={newton[-1]} "
              f"{lat[-1]:.1f} ms", file=sys.stderr, flush=True)
    taccel.device_synchronize()
    dt = time.perf_counter() - t0
    taccel.profile_enable(False)
    out = dict(
        metric=METRIC, value=ok / dt, unit="env-steps/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=dt * 1e3 / K, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64" if prec == taccel.FP64 else "f32+f64", data="synthetic",
        config=dict(workload=f"uniform batch of {n} small pads (243 verts, 768 tets) with "
                             "8-point hull indenters, pressed over 10 steps",
                    scenes=n, precision=args.precision, step_range=[W, W + K - 1],
                    friction=args.friction),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        roofline=_spmv_roofline(taccel),
    )
    b.close()
    return out


def run_serving(args, taccel, scenes, np):
    """Serving stream: Poisson arrivals, each request a 50-step rollout of a pad of random
    resolution with 1-3 hull indenters; continuous batching under an HBM budget."""
    import threading

    arrivals = scenes.serving_arrivals(args.rate, args.duration)
    print(f"generating {len(arrivals)} requests", file=sys.stderr, flush=True)
    reqs = [scenes.serving_request(i) for i in range(len(arrivals))]
    prec = taccel.MIXED if args.precision == "mixed" else taccel.FP64
    srv = taccel.Server(hbm_budget_bytes=args.budget_gb * 1e9, max_cohort=args.max_cohort,
                        max_cohorts=args.max_cohorts, coalesce_ms=2.0)
    ids = [None] * len(reqs)
    t0 = time.perf_counter()

    def feeder():
        for i, (ta, sp) in enumerate(zip(arrivals, reqs)):
            delay = ta - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ids[i] = srv.submit(sp, precision=prec)

    th = threading.Thread(target=feeder)
    th.start()
    done = {}
    last_print = time.perf_counter()
    while len(done) < len(reqs):
        for c in srv.poll(cap=256, wait_ms=100):
            done[c["req_id"]] = c
        if time.perf_counter() - last_print > 5:
            inf = srv.info()
            print(f"{time.perf_counter() - t0:.1f} s: {len(done)}/{len(reqs)} done, "
                  f"queued {inf['queued']}, cohorts {inf['running_cohorts']}, "
                  f"{inf['used_bytes'] / 1e9:.2f} GB", file=sys.stderr, flush=True)
            last_print = time.perf_counter()
    dt = time.perf_counter() - t0
    th.join()
    ok_steps = 0
    lat = []
    n_ok = 0
    for rid in ids:
        c = done[rid]
        good = c["steps_done"] - (0 if c["status"] == taccel.OK else 1)
        ok_steps += good
        n_ok += c["status"] == taccel.OK
        lat.extend(srv.step_latencies(rid).tolist())
    info = srv.info()
    srv.close()
    waits = [done[r]["wait_ms"] for r in ids]
    return dict(
        metric=METRIC, value=ok_steps / dt, unit="env-steps/s", n_gpus=1, steps=len(reqs),
        warmup=0, ms_per_step=float(np.mean(lat)), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64" if prec == taccel.FP64 else "f32+f64", data="synthetic",
        config=dict(workload=f"serving stream: Poisson {args.rate}/s for {args.duration} s, "
                             "50-step rollouts of pads {16x12x4, 32x24x6, 48x36x8} with 1-3 "
                             "hull indenters of 200-8000 tris",
                    requests=len(reqs), budget_gb=args.budget_gb, precision=args.precision,
                    max_cohort=args.max_cohort, max_cohorts=args.max_cohorts),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        requests_ok=n_ok, wall_s=dt, peak_device_gb=info["peak_bytes"] / 1e9,
        wait_p50_ms=float(np.percentile(waits, 50)), wait_p99_ms=float(np.percentile(waits, 99)),
        roofline=None,
    )


def run_tactile(args, taccel, scenes, np):
    """Tactile outputs of the benchmark pad after two press steps: a 640x480 depth and normal
    map of its coated face (1,536 triangles) at 50 um, and 1,200 markers, per call (each call
    includes the readback of its outputs to host memory)."""
    MM = scenes.MM
    spec = scenes.pad_press_slide_hull(0)
    sc = taccel.Scene(spec)
    for k in range(2):
        if sc.step(k)[0] != taccel.OK:
            sys.exit("tactile workload: press step failed")
    tris = scenes.top_surface_tris(spec)
    idx, bary = scenes.marker_layout(spec, tris, 40, 30)
    cam = taccel.camera((-16 * MM, -12 * MM, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.05 * MM,
                        640, 480)
    for _ in range(args.warmup):
        sc.depth_map(cam, tris)
        sc.markers(tris[idx], bary)
    taccel.device_synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sc.depth_map(cam, tris)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        sc.markers(tris[idx], bary)
    t2 = time.perf_counter()
    sc.close()
    K = args.steps
    return dict(metric="depth+normal maps per second (640x480, incl. readback)",
                value=K / (t1 - t0), unit="maps/s", n_gpus=1, steps=K, warmup=args.warmup,
                ms_per_step=(t1 - t0) * 1e3 / K, higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload="coated face of the 32x24x6 pad (1536 triangles), 640x480 "
                                     "orthographic depth and normal map at 50 um; 1200 markers"),
                markers_ms_per_call=(t2 - t1) * 1e3 / K)


def run_copy(args, taccel, scenes, np):
    """Counter calibration: three device-to-device copies of 256 MiB (a plain copy kernel of
    known size) through the HIP runtime."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    n = 256 << 20
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    for ptr in (a, b):
        if hip.hipMalloc(ctypes.byref(ptr), ctypes.c_size_t(n)) != 0:
            sys.exit("hipMalloc failed")
    if hip.hipMemset(a, 1, ctypes.c_size_t(n)) != 0:
        sys.exit("hipMemset failed")
    t0 = time.perf_counter()
    for _ in range(3):
        if hip.hipMemcpy(b, a, ctypes.c_size_t(n), 3) != 0:  # device to device
            sys.exit("hipMemcpy failed")
    hip.hipDeviceSynchronize()
    dt = time.perf_counter() - t0
    hip.hipFree(a)
    hip.hipFree(b)
    return dict(metric="device copy bandwidth (counter calibration)", value=3 * 2 * n / dt / 1e9,
                unit="GB/s", n_gpus=1, steps=3, warmup=0, ms_per_step=dt * 1e3 / 3,
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="u8",
                data="synthetic", config=dict(workload="copy 256 MiB device to device x3",
                                              bytes_per_copy=n))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["single", "batch", "serving", "tactile", "copy"],
                    default="single")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--scenes", type=int, default=64)
    ap.add_argument("--friction", type=float, default=0.0,
                    help="friction coefficient of the single/batch workload (default 0: the "
                         "frictionless benchmark)")
    ap.add_argument("--phases", type=int, default=0,
                    help="extra steps after the timed region with per-phase host timing")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=1.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-cohort", type=int, default=64)
    ap.add_argument("--max-cohorts", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (scenes would shard across GPUs without "
              "communication; there is no multi-GPU run)", file=sys.stderr)
        sys.exit(1)
    import numpy as np

    from paper_2504_12908_amd import scenes, taccel

    run = dict(single=run_single, batch=run_batch, serving=run_serving, tactile=run_tactile,
               copy=run_copy)[args.workload]
    out = run(args, taccel, scenes, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
