"""Benchmark: Newton-converged env-steps/s of the IPC time step on one MI355X.

Default workload (the batched form of the method, FP64): 256 independent copies of the small
gel pad (20x20x4 mm, 8x8x2 hex grid split into 6 tets per hex: 243 vertices, 768 tets, bottom
face fixed, neo-Hookean E = 0.3 MPa, nu = 0.45, rho = 1000), each pressed by its own seeded
rigid convex hull (8 points, 10 mm extent, rho = 2000) placed at an xy offset U(-3, 3) mm,
0.05 mm above the pad, and lowered to a press depth U(0.3, 1.2) mm over 10 steps; h = 0.01 s,
dhat = 1e-4 m, kappa = 1e3, Newton tolerance 1e-6.  Synthetic seeded input.  One launch per
stage covers all scenes.

A step is one call of taccel_batch_step (predict, Newton loops with broad phase, narrow phase,
barrier / FEM / affine-body derivatives, assembly, PCG, CCD, line search, augmented
Lagrangian rounds and snap, velocity update) for every scene.  After W warm-up steps the batch
is reset to its creation state and K steps are timed with the device synchronised on both
sides: the 10-step trajectory from its start, repeated (with a reset, inside the timed region)
when K > 10.  Only Newton-converged scene-steps count.

Beside it, in the same process:
* plain FP64 one scene at a time: the first scenes of the same batch, each stepped alone
  through its whole trajectory (vs_baseline is the ratio to this rate);
* the benchmark pad alone (32x24x6 grid, 5,775 vertices, 27,648 tets, pressed 1 mm and slid
  2 mm by a 796-triangle hull over 100 steps, h = 0.005 s), FP64, whole trajectory;
* roofline: the PCG sparse-product kernel timed with HIP events on the solver's stream, in a
  separate pass over the same trajectory after the timed region (the timing adds launches and
  synchronisations, so it stays out of the timed steps);
* cpu_baseline: the CPU FP64 oracle on the host's cores, one scene per thread.
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


def _host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(specs, max_threads=16, budget_s=30.0):
    """The oracle on the host, one scene per thread (ctypes releases the GIL), each scene
    stepped through its whole script; bounded to about budget_s of wall time."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import binding as O

    model, avail = _host_cpu()
    threads = max(1, min(avail, max_threads, len(specs)))
    t_stop = time.perf_counter() + budget_s

    def run(sp):
        o = O.OracleScene(sp)
        ok = 0
        for k in range(sp.n_steps):
            if time.perf_counter() > t_stop:
                break
            rc, _ = o.step(k)
            if rc != 0:
                break
            ok += 1
        return ok

    O.lib()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        oks = list(ex.map(run, specs[:threads]))
    dt = time.perf_counter() - t0
    return dict(value=sum(oks) / dt, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"scenes 0..{threads - 1} of the same workload, one per thread, each "
                       f"from its first step ({sum(oks)} scene-steps in {dt:.1f} s)",
                cpu_model=model, host_cpus_available=avail)


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


def _precision(args, taccel):
    """The --precision flag as the library's taccel_precision and the bench line's dtype."""
    return {"fp64": (taccel.FP64, "f64"), "mixed": (taccel.MIXED, "f32+f64"),
            "refined": (taccel.FP64_REFINED, "f64+f32")}[args.precision]


def _set_friction(args, specs):
    """--friction MU: the workload with the lagged friction potential (eps_v = 1e-3 m/s);
    --pcg-forcing 1: PCG tolerances by forcing terms."""
    for sp in specs:
        sp.params["pcg_forcing"] = args.pcg_forcing
    if args.friction > 0.0:
        for sp in specs:
            sp.params["friction"] = args.friction
            sp.params["eps_v"] = 1e-3


def _roofline_pass(taccel, step_fn, n_steps):
    """The sparse-product kernel timed with HIP events on the solver's stream over a separate
    pass of n_steps steps (after the timed region)."""
    taccel.device_synchronize()
    taccel.profile_reset()
    taccel.profile_enable(True)
    for k in range(n_steps):
        step_fn(k)
    taccel.device_synchronize()
    taccel.profile_enable(False)
    roof = _spmv_roofline(taccel)
    pcg = taccel.profile_query("pcg")
    if pcg["launches"]:
        roof["pcg_us_per_iter"] = pcg["total_ms"] * 1e3 / pcg["launches"]
    roof["measured_over"] = f"steps 0..{n_steps - 1} of the trajectory, after the timed region"
    return roof


def _refine_ratio(taccel, spec, prec, steps=3):
    """FP32 passes per Newton direction over the first steps of one scene (FP64_REFINED), in a
    pass of its own after the timed region."""
    sc = taccel.Scene(spec, precision=prec)
    taccel.profile_reset()
    taccel.profile_enable(True)
    for k in range(min(steps, spec.n_steps)):
        sc.step(k)
    taccel.profile_enable(False)
    sc.close()
    r = taccel.profile_query("refine")
    return r["launches"] / r["bytes"] if r["bytes"] else None


def _single_trajectory(taccel, spec, prec, log=None):
    """One scene stepped alone through its whole script (FP64 unless prec says otherwise);
    returns (Newton-converged steps, seconds, per-step latencies in ms, stats)."""
    sc = taccel.Scene(spec, precision=prec)
    taccel.device_synchronize()
    ok, lat, stats = 0, [], []
    t0 = time.perf_counter()
    for k in range(spec.n_steps):
        ts = time.perf_counter()
        rc, st = sc.step(k)
        lat.append((time.perf_counter() - ts) * 1e3)
        stats.append(st)
        if log:
            print(f"{log} step {k}: {taccel.STATUS_NAMES[rc]} newton={st['newton_iters']} "
                  f"al={st['al_rounds']} pcg={st['pcg_iters']} {lat[-1]:.1f} ms",
                  file=sys.stderr, flush=True)
        if rc != taccel.OK:
            break
        ok += 1
    taccel.device_synchronize()
    dt = time.perf_counter() - t0
    sc.close()
    return ok, dt, lat, stats


def run_single(args, taccel, scenes, np):
    """The benchmark pad alone (5,775 vertices, 796-triangle hull), its whole 100-step press
    and slide trajectory timed after a warm-up scene of W steps."""
    spec = scenes.pad_press_slide_hull(0)
    _set_friction(args, [spec])
    prec, dtype = _precision(args, taccel)
    if args.warmup > 0:
        warm = taccel.Scene(spec, precision=prec)
        for k in range(min(args.warmup, spec.n_steps)):
            warm.step(k)
        warm.close()
    ok, dt, lat, stats = _single_trajectory(taccel, spec, prec, log="single")
    n = len(lat)
    out = dict(
        metric=METRIC, value=ok / dt, unit="env-steps/s", n_gpus=1, steps=n, warmup=args.warmup,
        ms_per_step=dt * 1e3 / n, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=dtype, data="synthetic",
        config=dict(workload="gel pad 32x24x6 grid (5775 verts, 27648 tets) pressed 1 mm and "
                             "slid 2 mm by a 400-point convex hull (796 tris), 1 scene, whole "
                             "100-step trajectory",
                    scenes=1, h=spec.params["h"], precision=args.precision,
                    friction=args.friction, pcg_forcing=args.pcg_forcing),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        newton_iters_per_step=float(np.mean([s["newton_iters"] for s in stats])),
        pcg_iters_per_step=float(np.mean([s["pcg_iters"] for s in stats])),
    )
    sc = taccel.Scene(spec, precision=prec)
    out["roofline"] = _roofline_pass(taccel, lambda k: sc.step(k), min(args.roofline_steps, spec.n_steps))
    sc.close()
    if args.phases > 0:
        # host wall time of each Newton-iteration phase over the first steps (every phase ends
        # with a synchronisation here, so the sum exceeds an unprofiled iteration)
        sc = taccel.Scene(spec, precision=prec)
        taccel.profile_reset()
        taccel.profile_enable(False, phases=True)
        for k in range(min(args.phases, spec.n_steps)):
            sc.step(k)
        taccel.profile_enable(False)
        sc.close()
        ph = {name: taccel.profile_query(name) for name in taccel.PHASES}
        n_it = max(ph["solve"]["launches"], 1)
        out["phase_ms_per_newton_iter"] = {name: v["total_ms"] / n_it for name, v in ph.items()}
    if prec == taccel.FP64:
        out["roofline"]["traffic"] = _measured_traffic()
    if prec == taccel.FP64_REFINED:
        out["fp32_passes_per_direction"] = _refine_ratio(taccel, spec, prec)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline([spec], budget_s=args.cpu_budget)
    return out


def run_batch(args, taccel, scenes, np):
    """Uniform batch: n copies of the small pad with seeded hull indenters, one launch per
    stage over all scenes; the whole trajectory timed from its start."""
    n = args.scenes
    if n > 1024:
        sys.exit("bench.py: batches of more than 1,024 scenes are off: a 4,096-scene batch "
                 "once ended in a GPU memory fault whose cause is not shown")
    specs = scenes.uniform_batch(n)
    _set_friction(args, specs)
    nst = specs[0].n_steps
    W, K = args.warmup, args.steps
    prec, dtype = _precision(args, taccel)
    if prec == taccel.MIXED and n > 1:
        sys.exit("bench.py: mixed precision runs one scene per batch (see include/taccel.h)")
    t_create = time.perf_counter()
    b = taccel.Batch(specs, precision=prec)
    t_create = time.perf_counter() - t_create
    print(f"batch of {n} created in {t_create:.2f} s", file=sys.stderr, flush=True)
    targets = [b.targets(k) for k in range(nst)]
    for k in range(W):
        rc, per, st = b.step(k % nst, targets[k % nst])
        print(f"warmup step {k % nst}: ok={int((per == taccel.OK).sum())}/{n} "
              f"{st[0]['step_ms']:.1f} ms", file=sys.stderr, flush=True)
    b.reset()
    taccel.device_synchronize()
    lat, ok, newton, per_ok = [], 0, [], np.zeros(n, dtype=np.int64)
    t0 = time.perf_counter()
    for i in range(K):
        k = i % nst
        ts = time.perf_counter()
        if i > 0 and k == 0:
            b.reset()
        rc, per, st = b.step(k, targets[k])
        lat.append((time.perf_counter() - ts) * 1e3)
        good = per == taccel.OK
        ok += int(good.sum())
        per_ok += good
        newton.append(max(s["newton_iters"] for s in st))
        print(f"step {k}: ok={int(good.sum())}/{n} max_newton={newton[-1]} "
              f"mean_newton={np.mean([s['newton_iters'] for s in st]):.1f} {lat[-1]:.1f} ms",
              file=sys.stderr, flush=True)
    taccel.device_synchronize()
    dt = time.perf_counter() - t0
    value = ok / dt
    out = dict(
        metric=METRIC, value=value, unit="env-steps/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=dt * 1e3 / K, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=dtype, data="synthetic",
        config=dict(workload=f"uniform batch of {n} small pads (243 verts, 768 tets each) with "
                             "seeded 8-point hull indenters, pressed over the whole 10-step "
                             "trajectory", scenes=n, precision=args.precision,
                    steps_per_trajectory=nst, friction=args.friction,
                    pcg_forcing=args.pcg_forcing),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        scene_steps_ok=ok, scene_steps=n * K, max_newton_per_step=int(max(newton)),
        create_s=t_create,
    )
    # plain FP64, one scene at a time: the first scenes of the same batch, whole trajectories
    m = max(1, min(args.plain_scenes, n))
    plain_ok, plain_dt = 0, 0.0
    if m > 0:
        import copy
        plain_specs = []
        for sp in specs[:m]:  # plain: FP64 at the fixed PCG tolerance
            sp2 = copy.copy(sp)
            sp2.params = dict(sp.params, pcg_forcing=0)
            plain_specs.append(sp2)
        warm = taccel.Scene(plain_specs[0])
        warm.step(0)
        warm.close()
        for sp in plain_specs:
            o_, d_, _, _ = _single_trajectory(taccel, sp, taccel.FP64)
            plain_ok += o_
            plain_dt += d_
    plain = plain_ok / plain_dt if plain_dt > 0 else None
    out["plain_fp64_one_at_a_time"] = dict(
        value=plain, unit="env-steps/s", scenes=m,
        sample=f"scenes 0..{m - 1} of the batch, each alone (taccel_step, FP64) through its "
               f"{nst}-step trajectory")
    out["vs_baseline"] = value / plain if plain else None
    b.reset()
    out["roofline"] = _roofline_pass(taccel, lambda k: b.step(k, targets[k]), nst)
    b.close()
    if args.c2:
        spec = scenes.pad_press_slide_hull(0)
        o_, d_, lat2, _ = _single_trajectory(taccel, spec, taccel.FP64)
        out["single_benchmark_pad_fp64"] = dict(
            value=o_ / d_, unit="env-steps/s", steps_ok=o_, p50_ms=float(np.percentile(lat2, 50)),
            p99_ms=float(np.percentile(lat2, 99)),
            workload="gel pad 32x24x6 grid (5775 verts) pressed and slid by a 796-triangle "
                     "hull, whole 100-step trajectory, alone")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(specs, budget_s=args.cpu_budget)
        v = out["cpu_baseline"]["value"]
        out["cpu_baseline"]["gpu_over_cpu"] = value / v if v > 0 else None
    return out


def run_grasp(args, taccel, scenes, np):
    """Two-finger grasp and lift (two 5,775-vertex pads on the fingers of a parallel gripper
    driven by forward kinematics, a free 10,000-triangle hull held by friction), n scenes in
    one batch; the first K steps of the 200-step trajectory timed.  With --precision mixed the
    batch is one scene (mixed batches of several scenes are refused), and the line also gives
    the mixed path's error against the FP64 path, step by step from the FP64 state."""
    n = args.scenes
    prec, dtype = _precision(args, taccel)
    if prec == taccel.MIXED and n > 1:
        sys.exit("bench.py: mixed precision runs one scene per batch (see include/taccel.h)")
    specs = [scenes.grasp_lift(i) for i in range(n)]
    W, K = args.warmup, args.steps
    nst = specs[0].n_steps
    if K > nst:
        sys.exit(f"steps must be <= {nst}")
    b = taccel.Batch(specs, precision=prec)
    targets = [b.targets(k) for k in range(K)]
    for k in range(min(W, K)):
        b.step(k, targets[k])
    b.reset()
    ref = taccel.Batch(specs) if prec == taccel.MIXED else None
    taccel.device_synchronize()
    lat, ok = [], 0
    err = 0.0
    t0 = time.perf_counter()
    for k in range(K):
        ts = time.perf_counter()
        rc, per, st = b.step(k, targets[k])
        lat.append((time.perf_counter() - ts) * 1e3)
        ok += int((per == taccel.OK).sum())
        print(f"step {k}: ok={int((per == taccel.OK).sum())}/{n} "
              f"max_newton={max(s['newton_iters'] for s in st)} {lat[-1]:.1f} ms",
              file=sys.stderr, flush=True)
    taccel.device_synchronize()
    dt = time.perf_counter() - t0
    if ref is not None:
        # per step from a common start: the mixed scene takes the FP64 scene's state first
        for k in range(K):
            for f in (taccel.FIELD_X, taccel.FIELD_V, taccel.FIELD_Q, taccel.FIELD_QDOT):
                b.write(0, f, ref.read(0, f))
            b.step(k, targets[k])
            ref.step(k, targets[k])
            err = max(err, float(np.abs(b.read(0, taccel.FIELD_X) - ref.read(0, taccel.FIELD_X)).max()))
        ref.close()
    out = dict(
        metric=METRIC, value=ok / dt, unit="env-steps/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=dt * 1e3 / K, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=dtype, data="synthetic",
        config=dict(workload=f"two-finger grasp and lift, {n} scene(s): two 32x24x6-cell pads "
                             "(11,550 verts, 55,296 tets) on gripper links, a free 10,000-triangle "
                             "hull held by friction; first steps of the 200-step trajectory",
                    scenes=n, precision=args.precision),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
    )
    if ref is not None:
        out["mixed_vs_fp64_max_abs_m"] = err
        out["mixed_tolerance_m"] = 1e-4 * 6e-3
    b.close()
    return out


def run_serving(args, taccel, scenes, np):
    """Serving stream: Poisson arrivals, each request a 50-step rollout of a pad of random
    resolution with 1-3 hull indenters; continuous batching under an HBM budget."""
    import threading

    arrivals = scenes.serving_arrivals(args.rate, args.duration)
    print(f"generating {len(arrivals)} requests", file=sys.stderr, flush=True)
    reqs = [scenes.serving_request(i) for i in range(len(arrivals))]
    prec, dtype = _precision(args, taccel)
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
    plain = None
    if args.comparator:
        # the same requests solved one at a time, each scene alone, FP64, in arrival order
        t1 = time.perf_counter()
        p_ok, p_lat, p_req_ok = 0, [], 0
        for sp in reqs:
            sc = taccel.Scene(sp)
            good = 0
            for k in range(sp.n_steps):
                ts = time.perf_counter()
                rc, _ = sc.step(k)
                p_lat.append((time.perf_counter() - ts) * 1e3)
                if rc != taccel.OK:
                    break
                good += 1
            sc.close()
            p_ok += good
            p_req_ok += good == sp.n_steps
        pdt = time.perf_counter() - t1
        plain = dict(value=p_ok / pdt, unit="env-steps/s", requests_ok=p_req_ok, wall_s=pdt,
                     p50_ms=float(np.percentile(p_lat, 50)), p99_ms=float(np.percentile(p_lat, 99)),
                     sample="the same requests, each scene alone with taccel_step in FP64, one "
                            "after another")
    return dict(
        metric=METRIC, value=ok_steps / dt, unit="env-steps/s", n_gpus=1, steps=len(reqs),
        warmup=0, ms_per_step=float(np.mean(lat)), higher_is_better=True, scaling="weak",
        dtype=dtype, data="synthetic",
        config=dict(workload=f"serving stream: Poisson {args.rate}/s for {args.duration} s, "
                             "50-step rollouts of pads {16x12x4, 32x24x6, 48x36x8} with 1-3 "
                             "hull indenters of 200-8000 tris",
                    requests=len(reqs), budget_gb=args.budget_gb, precision=args.precision,
                    max_cohort=args.max_cohort, max_cohorts=args.max_cohorts),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        requests_ok=n_ok, wall_s=dt, peak_device_gb=info["peak_bytes"] / 1e9,
        wait_p50_ms=float(np.percentile(waits, 50)), wait_p99_ms=float(np.percentile(waits, 99)),
        roofline=None, plain_fp64_one_at_a_time=plain,
        vs_baseline=(ok_steps / dt) / plain["value"] if plain and plain["value"] > 0 else None,
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
    ap.add_argument("--workload", choices=["single", "batch", "grasp", "serving", "tactile", "copy"],
                    default="batch")
    ap.add_argument("--precision", choices=["fp64", "mixed", "refined"], default="fp64",
                    help="fp64; mixed (FP32 Hessians, SpMV and PCG); refined (FP64 system, FP32 "
                         "PCG passes with FP64 residual refinement)")
    ap.add_argument("--scenes", type=int, default=256)
    ap.add_argument("--plain-scenes", type=int, default=16,
                    help="scenes of the batch also stepped one at a time (FP64 comparator)")
    ap.add_argument("--roofline-steps", type=int, default=10,
                    help="steps of the separate sparse-product timing pass (single workload)")
    ap.add_argument("--cpu-budget", type=float, default=30.0,
                    help="seconds of the oracle's host run (cpu_baseline)")
    ap.add_argument("--no-c2", dest="c2", action="store_false",
                    help="skip the benchmark pad's one-scene trajectory beside the batch")
    ap.add_argument("--friction", type=float, default=0.0,
                    help="friction coefficient of the single/batch workload (default 0: the "
                         "frictionless benchmark)")
    ap.add_argument("--pcg-forcing", type=int, choices=[0, 1], default=0,
                    help="single/batch: 1 = PCG tolerance per Newton iteration by Eisenstat-Walker "
                         "forcing terms (default 0: the fixed tolerance)")
    ap.add_argument("--phases", type=int, default=0,
                    help="single workload: steps of a separate pass with per-phase host timing")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=1.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-cohort", type=int, default=64)
    ap.add_argument("--max-cohorts", type=int, default=4)
    ap.add_argument("--no-comparator", dest="comparator", action="store_false",
                    help="serving: skip solving the same requests one at a time in FP64")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (scenes would shard across GPUs without "
              "communication; there is no multi-GPU run)", file=sys.stderr)
        sys.exit(1)
    import numpy as np

    from paper_2504_12908_amd import scenes, taccel

    run = dict(single=run_single, batch=run_batch, grasp=run_grasp, serving=run_serving,
               tactile=run_tactile, copy=run_copy)[args.workload]
    out = run(args, taccel, scenes, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
