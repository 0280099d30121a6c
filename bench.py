#!/usr/bin/env python3
"""Throughput of the coupled TLED + Pennes step on one MI355X.

One step = one pass of the whole hot path (element physics, assembly, node
updates) over the ~1.0M-tet noisy-ellipsoid workload (0.2 x 0.15 x 0.1 m,
~180k nodes, two Prony terms, shrinkage, 1/r^4 line source).  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--variant 1|2] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per element-update of the dominant kernel: connectivity
# 4 or 8 ints, dh/dX (3 or 7 rows of 3 floats), V0, fibre (3 floats), H8
# hourglass vectors and stiffness (29 floats), Prony state read and written
# (24 B per term each way); plus 73 B per node of node state advanced inside it.
def elem_bytes(npe: int, n_prony: int) -> float:
    if npe == 4:
        return 16 + 36 + 4 + 12 + 48.0 * n_prony
    return 32 + 84 + 4 + 12 + 116 + 48.0 * n_prony


NODE_BYTES = 73.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--variant", type=int, default=0, help="kernel variant (0: the library default)")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="steps per hipGraph chunk (0: library default, 50 for a problem, eager steps for a batch)")
    ap.add_argument("--patch-elems", type=int, default=0, help="elements per patch (0: library default)")
    ap.add_argument("--block-size", type=int, default=0, help="patch kernel threads per workgroup (0: default)")
    ap.add_argument("--thermal-dose", action="store_true",
                    help="accumulate CEM43 and the Arrhenius integral per node (a published liver set, "
                         "A = 7.39e39 /s, Ea = 2.577e5 J/mol) and report the damaged volumes")
    ap.add_argument("--shared-update", type=int, default=0, choices=[0, 1, 2],
                    help="shared nodes advanced inside the next step's patch kernel (1, the default where "
                         "available) or by a kernel of their own after every step (2)")
    ap.add_argument("--reorder", type=int, default=0,
                    help="element order: 0/1 Morton with bisection patches, 2 Morton runs, -1 as generated")
    ap.add_argument("--elems", type=int, default=1_000_000)
    ap.add_argument("--workload", default="ellipsoid_t4", choices=["ellipsoid_t4", "cube_h8", "cube_t4"],
                    help="ellipsoid_t4: ~1.0M-tet noisy ellipsoid (default); cube_h8: 64^3 H8 cube; "
                         "cube_t4: the 6000-tet parity cube (cache-resident, launch-bound)")
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed regions of --steps steps each; value is their median, all are reported")
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle steps for the CPU baseline (0: auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", type=int, default=0, metavar="N",
                    help="instead of the headline run: batched planning sweep of N scenarios (one JSON line)")
    ap.add_argument("--duration-scale", type=float, default=1e-3,
                    help="sweep heating durations are U(30, 300) s times this factor")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--schedule", default="auto", choices=["auto"] + ["prefix-eager", "prefix-graph-50",
                                                                        "persistent-graph-100", "persistent-graph-400"],
                    help="batch launch schedule of the sweep (auto: chosen by the autotuner)")
    ap.add_argument("--surrogate", type=int, default=0, metavar="N_TRAIN",
                    help="instead of the headline run: train the surrogate ensemble on N_TRAIN planning runs and "
                         "compare scenarios/s of surrogate-with-fallback against the solver (one JSON line)")
    ap.add_argument("--holdout", type=int, default=200)
    ap.add_argument("--data-dir", default="",
                    help="surrogate training data: with --shard, where to write it; else, if it holds shards "
                         "of the N_TRAIN training runs, train on them instead of solving the runs here")
    ap.add_argument("--shard", default="", metavar="K/N",
                    help="with --surrogate N_TRAIN: only solve the K-th of N slices of the training runs and "
                         "store a node subsample of their snapshots in --data-dir (training data made in "
                         "separate runs)")
    ap.add_argument("--shard-nodes", type=int, default=2048, help="nodes stored per snapshot field")
    ap.add_argument("--surrogate-schedule", type=int, default=0, choices=[0, 1],
                    help="batch schedule of the surrogate's solver runs (1: persistent kernels in graph chunks of 100)")
    ap.add_argument("--calib", type=int, default=100, help="solver runs held back to calibrate the disagreement")
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--members", type=int, default=4)
    ap.add_argument("--snapshots", type=int, default=5)
    ap.add_argument("--threshold", type=float, default=0.5, help="K")
    ap.add_argument("--train-batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--sigma", type=float, default=1.0, help="Fourier frequency standard deviation")
    ap.add_argument("--counters-summary", nargs=6, default=None,
                    metavar=("WORKLOAD", "FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB", "COPY_MIB"),
                    help="write profiles/traffic_WORKLOAD.json from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE "
                         "databases of a bench run and of a --copy-calibration run")
    ap.add_argument("--step-time-profile", action="store_true",
                    help="per-region step time of the T4 ellipsoid along a run: 100 back-to-back regions of "
                         "--steps steps from a fresh process, the same again from the initial state, 40 "
                         "regions each after 5 ms of idle, one region of 2000 steps, then 30 regions from the "
                         "initial state again")
    ap.add_argument("--mlp-train-timing", action="store_true",
                    help="time training steps of the surrogate network (width 256, depth 5, 16384 random "
                         "samples), fused forward against the layer-by-layer GEMMs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 launches) to calibrate HBM counters")
    return ap.parse_args()


def copy_calibration(mib: int):
    """The library's plain streaming copy kernel at a known size: its FETCH_SIZE / WRITE_SIZE give
    the counter scale."""
    import torch
    from paper_2009_10400_amd import tled
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        tled.stream_copy(dst, src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 5, "kernel": "stream_copy_kernel"}), flush=True)


def _counter_means(db_path: str, counter: str):
    """Mean value per dispatch of one counter, per kernel name, from a rocprofv3 database."""
    import sqlite3
    con = sqlite3.connect(db_path)
    rows = con.execute("select kernel_name, avg(value), count(*) from "
                       "(select dispatch_id, kernel_name, sum(value) as value from counters_collection "
                       " where counter_name = ? group by dispatch_id, kernel_name) group by kernel_name",
                       (counter,)).fetchall()
    con.close()
    return {k: (v, n) for k, v, n in rows}


def workload_key(name: str, elems: int) -> str:
    """Name of a measured workload: the T4 ellipsoid at other than 1M elements carries its size."""
    return name if name != "ellipsoid_t4" or elems == 1_000_000 else f"{name}_{elems}"


def problem_for_key(key: str):
    from paper_2009_10400_amd import workloads as W
    if key == "cube_h8":
        return W.cube_h8(64)
    size = key[len("ellipsoid_t4_"):] if key.startswith("ellipsoid_t4_") else "1000000"
    return W.ellipsoid_t4(int(size))


def counters_summary(workload, fetch_db, write_db, copy_fetch_db, copy_write_db, copy_mib):
    """HBM traffic of the dominant kernel per launch: FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what the counter reads for a plain device copy of known size."""
    from paper_2009_10400_amd import tled, workloads as W
    from paper_2009_10400_amd.build import source_digest
    copy_bytes = int(copy_mib) * (1 << 20)
    cf = max(_counter_means(copy_fetch_db, "FETCH_SIZE").items(), key=lambda kv: kv[1][0])
    cw = max(_counter_means(copy_write_db, "WRITE_SIZE").items(), key=lambda kv: kv[1][0])
    fetch_scale = copy_bytes / (cf[1][0] * 1024.0)
    write_scale = copy_bytes / (cw[1][0] * 1024.0)
    f = _counter_means(fetch_db, "FETCH_SIZE")
    w = _counter_means(write_db, "WRITE_SIZE")

    def pick(d, name, second=False):
        """The instantiation of the kernel with the most dispatches (the steady-state one), or
        with second=True the one with the next most (None if there is none)."""
        ks = sorted((k for k in d if f"{name}<" in k), key=lambda k: -d[k][1])
        if second:
            return d[ks[1]] if len(ks) > 1 else None
        return d[ks[0]]

    fk, nd = pick(f, "patch_kernel")
    wk, _ = pick(w, "patch_kernel")
    sf, _ = pick(f, "shared_node_kernel")
    sw, _ = pick(w, "shared_node_kernel")
    p = problem_for_key(workload)
    h = tled.from_problem(p, device=-1)
    info = h.info()
    h.close()
    fused = info["shared_update"] == 1
    # a fused launch advances every node (its patch's interior nodes by this step, its shared
    # nodes by the previous one); an unfused one the interior nodes only
    alg = elem_bytes(p.npe, info["n_prony"]) * p.ne + NODE_BYTES * (
        info["n_nodes"] if fused else info["n_nodes"] - info["n_shared_nodes"])
    first = None
    if fused:   # the first step of each chunk runs the unfused patch kernel
        f2, w2 = pick(f, "patch_kernel", True), pick(w, "patch_kernel", True)
        if f2 is not None and w2 is not None:
            first = [f2[0], w2[0]]
    out = {"kernel": "patch_kernel", "workload": workload, "source_digest": source_digest(),
           "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "fetch_scale": fetch_scale,
           "write_scale": write_scale,
           "bytes_per_launch": fk * 1024.0 * fetch_scale + wk * 1024.0 * write_scale,
           "algorithmic_bytes_per_launch": alg, "dispatches": nd,
           "layout": {"kernel_variant": info["kernel_variant"], "n_patches": info["n_patches"],
                      "n_shared_nodes": info["n_shared_nodes"], "shared_update": info["shared_update"]},
           "shared_node_kernel_kib": [sf, sw],
           "chunk_first_patch_kernel_kib": first,
           "note": f"scales from a plain {copy_mib} MiB device copy (FETCH_SIZE read {cf[1][0]:.1f} KiB, "
                   f"WRITE_SIZE {cw[1][0]:.1f} KiB)"}
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def traffic_record(workload: str, info=None):
    """The committed rocprofv3 counter summary of the solver kernels, if it is current: same
    solver sources, and (given the run's ``info``) the same patch layout as the counted run."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        from paper_2009_10400_amd.build import source_digest
        if d.get("source_digest") != source_digest():
            return None
        if info is not None:
            lay = d.get("layout", {})
            if any(lay.get(k) != info[k] for k in ("kernel_variant", "n_patches", "n_shared_nodes",
                                                    "shared_update")):
                return None
        return d
    except Exception:  # noqa: BLE001
        return None


def traffic_from_profiles(kernel_name: str, workload: str, info=None):
    """HBM bytes per launch of the dominant kernel from the counter summary, if it is current."""
    d = traffic_record(workload, info)
    if d is None or d.get("kernel") != kernel_name:
        return None
    return float(d["bytes_per_launch"])


def copy_bandwidth(mib: int = 1024, reps: int = 5):
    """GB/s of the library's plain streaming copy kernel (read + write bytes / time), HIP events
    recorded on the stream the copies run on."""
    import torch
    from paper_2009_10400_amd import tled
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    st = torch.cuda.Stream(device=0)
    with torch.cuda.stream(st):
        tled.stream_copy(dst, src, st.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            tled.stream_copy(dst, src, st.cuda_stream)
        e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(dst, src))
    del src, dst
    if not ok:
        raise RuntimeError("stream copy produced wrong data")
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def mlp_train_timing(args):
    """Training-step time of the surrogate network on random data: the forward pass through the
    fused kernel (default) and through the layer-by-layer GEMMs, HIP-event GEMM time included."""
    import torch
    from paper_2009_10400_amd import surrogate as S
    dev = torch.device("cuda", 0)
    n = args.train_batch
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.uniform(-1, 1, (n, 3)).astype(np.float32)).to(dev)
    p = torch.from_numpy(rng.uniform(-1, 1, (n, 11)).astype(np.float32)).to(dev)
    t = torch.from_numpy(rng.normal(size=(n, 4)).astype(np.float32)).to(dev)
    out = {"metric": "surrogate training step", "samples_per_step": n,
           "net": "64 Fourier frequencies + 11 parameters -> 5 x 256 SiLU -> 4", "data": "synthetic"}
    for lw in (False, True):
        m = S.MLP(0, n_freq=64, width=256, depth=5, n_out=4, seed=3, layerwise=lw)
        for _ in range(10):
            m.train_step(x, p, t, 1e-4)
        m.set_timing(True)
        for _ in range(10):
            m.train_step(x, p, t, 1e-4)
        tm = m.timing()
        m.set_timing(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            m.train_step(x, p, t, 1e-4)
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t0) / 50 * 1e3
        key = "layer_by_layer" if lw else "fused_forward"
        out[key] = {"train_step_ms": step_ms, "gemm_us_per_step": tm["gemm_ms"] / 10 * 1e3,
                    "gemm_TFLOPs": tm["gemm_flops"] / (tm["gemm_ms"] * 1e-3) / 1e12}
        log(f"[mlp] {key}: {out[key]}")
        m.close()
    print(json.dumps(out), flush=True)


def step_time_profile(args):
    """How the time per step of a short timed region depends on the GPU's recent activity: regions
    of --steps steps (each bracketed by device synchronisation, as in the timed run), back to back
    from a fresh process, again from the same initial state once the GPU is busy, and with 5 ms
    of idle before each region."""
    import torch
    from paper_2009_10400_amd import tled, workloads as W
    p = W.ellipsoid_t4(args.elems)
    stream = torch.cuda.Stream(device=0)
    sim = tled.from_problem(p, device=0, stream=stream.cuda_stream, graph_steps=args.graph_steps)
    blob = sim.get_state()
    sim.prepare(args.steps)
    torch.cuda.synchronize()
    K = args.steps

    def regions(n, idle=0.0):
        us = []
        for _ in range(n):
            if idle:
                time.sleep(idle)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sim.step(K)
            torch.cuda.synchronize()
            us.append(round(1e6 * (time.perf_counter() - t1) / K, 2))
        return us

    out = {"metric": "time per step of a timed region of K steps (us)", "workload": p.name, "elements": p.ne,
           "K": K, "data": "synthetic"}
    out["fresh_process"] = regions(100)
    sim.set_state(blob)
    out["again_from_initial_state"] = regions(100)
    sim.set_state(blob)
    out["idle_5ms_before_each"] = regions(40, idle=0.005)
    t1 = time.perf_counter()
    sim.step(2000)
    torch.cuda.synchronize()
    out["one_region_of_2000_steps"] = round(1e6 * (time.perf_counter() - t1) / 2000, 2)
    sim.set_state(blob)
    out["from_initial_state_after_that_region"] = regions(30)
    for k in ("fresh_process", "again_from_initial_state", "idle_5ms_before_each",
              "from_initial_state_after_that_region"):
        v = out[k]
        log(f"[profile] {k}: first 5 {v[:5]}, median of the last half {float(np.median(v[len(v) // 2:])):.2f}")
    sim.close()
    print(json.dumps(out), flush=True)


def dose_summary(sim):
    """Thermal dose after the run: largest CEM43 and Arrhenius integral, and the lumped volumes
    past the usual thresholds (240 equivalent minutes, Omega = 1) beside the 60 C monitor."""
    cem, om = sim.read_thermal_dose()
    vols = sim.damage_volumes(240.0, 1.0)
    m = sim.monitors()
    return {"cem43_max_min": float(cem.max()), "omega_max": float(om.max()),
            "volume_cem43_240_m3": vols["cem43"], "volume_omega_1_m3": vols["arrhenius"],
            "volume_60C_m3": m["ablated_volume"], "T_max_K": m["T_max"], "simulated_s": m["t"],
            "arrhenius": {"A_per_s": 7.39e39, "Ea_J_per_mol": 2.577e5}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(problem, dt, steps):
    import oracle
    oracle.build()
    o = oracle.OracleSim(problem.npe, problem.X, problem.conn, problem.params, a0=problem.a0, q=problem.q,
                         fix=problem.fix, t_on=problem.t_on, t_off=problem.t_off, dt=dt, gamma=problem.gamma)
    st = o.initial_state(problem.params["T0"])
    o.run(st, 1)                     # first touch of the state arrays
    t0 = time.perf_counter()
    o.run(st, steps)
    el = time.perf_counter() - t0
    return {"value": problem.ne * steps / el, "unit": "element-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the full {problem.ne}-tet workload, serial FP64 oracle ({el:.1f} s)",
            "cpu_model": cpu_model(), "host_cores_available": host_threads()}


def host_threads() -> int:
    """Host cores this process may use (its affinity), capped by OMP_NUM_THREADS when set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(cap))) if cap.isdigit() and int(cap) > 0 else n


def cpu_baseline_all_cores(problem, dt, steps, threads):
    """The same serial oracle on every host core at once: `threads` independent copies of the
    workload, each advanced `steps` steps by its own thread (the oracle's C calls release the
    GIL).  Throughput of the whole host, with the oracle's arithmetic unchanged."""
    import threading
    import oracle
    oracle.build()
    sims, states = [None] * threads, [None] * threads

    def make(i):
        o = oracle.OracleSim(problem.npe, problem.X, problem.conn, problem.params, a0=problem.a0, q=problem.q,
                             fix=problem.fix, t_on=problem.t_on, t_off=problem.t_off, dt=dt, gamma=problem.gamma)
        st = o.initial_state(problem.params["T0"])
        o.run(st, 1)
        sims[i], states[i] = o, st

    ths = [threading.Thread(target=make, args=(i,)) for i in range(threads)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    if any(o is None for o in sims):
        raise RuntimeError("oracle set-up failed")
    go = threading.Barrier(threads + 1)

    def work(i):
        go.wait()
        sims[i].run(states[i], steps)

    ths = [threading.Thread(target=work, args=(i,)) for i in range(threads)]
    for t in ths:
        t.start()
    go.wait()
    t0 = time.perf_counter()
    for t in ths:
        t.join()
    el = time.perf_counter() - t0
    return {"value": threads * problem.ne * steps / el, "unit": "element-updates/s", "cores": threads,
            "kind": "oracle, one independent copy per core",
            "sample": f"{threads} copies x {steps} steps of the full {problem.ne}-tet workload, serial FP64 "
                      f"oracle per thread ({el:.1f} s)"}


def sweep(args):
    """Batched planning sweep: N scenarios (5k-200k tets, log-uniform) in one batch, every scenario run
    to the end of its heating; reports scenarios/s and element-updates/s of the batch."""
    import torch
    from paper_2009_10400_amd import autotune, tled, workloads as W

    t = time.time()
    sc = W.planning_scenarios(args.sweep, seed=3, duration_scale=args.duration_scale)
    probs = [p for p, _ in sc]
    ne_tot = sum(p.ne for p in probs)
    log(f"[sweep] {len(sc)} scenarios, {ne_tot} elements, built in {time.time() - t:.1f}s")
    stream = torch.cuda.Stream(device=0)
    choice, report, sched_report = {}, {}, None
    if not args.no_autotune:
        t = time.time()
        choice, report = autotune.tune(probs, stream=stream.cuda_stream, log=log)
        log(f"[sweep] autotune {time.time() - t:.1f}s -> {choice}")
    if args.schedule == "auto":
        t = time.time()
        sched, sched_opts, sched_report = autotune.tune_schedule(probs, [d for _, d in sc], choice,
                                                                 stream=stream.cuda_stream, log=log)
        log(f"[sweep] schedule autotune {time.time() - t:.1f}s -> {sched}")
    else:
        sched, sched_opts = args.schedule, dict(autotune.SCHEDULES[args.schedule])
    if args.graph_steps:
        sched_opts["graph_steps"] = args.graph_steps
    t = time.time()
    b = tled.Batch(0, stream=stream.cuda_stream)
    b.set_options(**sched_opts)
    for p, dur in sc:
        b.add(p, cfl=p.cfl, t_end=dur, patch_elems=choice.get(autotune.bucket_of(p.ne), 0))
    b.finalize()
    steps = [b.scenario_steps(k)[1] for k in range(len(sc))]
    t_setup = time.time() - t
    log(f"[sweep] set-up (add + finalize) {t_setup:.1f}s, steps {min(steps)}..{max(steps)}, info={b.batch_info()}")
    torch.cuda.synchronize()
    # Batch steps are enqueued in chunks of about 20 s each, with a progress line per chunk (a
    # full-length sweep runs for minutes).  A scenario that goes unstable is reported, not dropped.
    t0 = time.perf_counter()
    nmax, done, chunk, status = max(steps), 0, 2000, "ok"
    try:
        while done < nmax:
            k = min(chunk, nmax - done)
            t1 = time.perf_counter()
            b.step(k)
            b.sync()
            done += k
            dt_chunk = time.perf_counter() - t1
            log(f"[sweep] {done}/{nmax} batch steps, {time.perf_counter() - t0:.1f}s")
            chunk = int(max(100, min(4 * chunk, k * 20.0 / max(dt_chunk, 1e-3))))
    except tled.TledError as e:
        status = str(e)
        log(f"[sweep] stopped at batch step {done}: {status}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    updates = sum(p.ne * min(n, done) for p, n in zip(probs, steps))
    tmax, vol, mon_status = b.scenario_monitors(333.15, strict=False)
    unstable = [k for k in range(len(sc)) if not np.isfinite(tmax[k])]
    per = [{"k": k, "kind": p.meta["kind"], "n_elems": int(p.ne), "n_nodes": int(p.nn),
            "dt": b.scenario_steps(k)[0], "steps": int(steps[k]), "heating_s": float(dur),
            "power_W": float(p.meta["power"]), "E_Pa": float(p.meta["E"]),
            "T_max_K": float(tmax[k]), "ablated_volume_m3": float(vol[k]), "finite": bool(np.isfinite(tmax[k]))}
           for k, ((p, dur), _) in enumerate(zip(sc, steps))]
    out = {
        "metric": "scenarios/s (batched planning sweep, solver)", "value": len(sc) / el, "unit": "scenarios/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "element_updates_per_s": updates / el, "seconds": el, "setup_seconds": t_setup, "batch_steps": max(steps),
        "config": {"workload": f"{len(sc)} scenarios, tet cubes and noisy ellipsoids of 5k-200k elements "
                               f"(log-uniform, {ne_tot} total), probe 1/r^2 source U(20,80) W, E U(2,6) kPa, "
                               f"heating U(30,300) s x {args.duration_scale:g}",
                   "duration_scale": args.duration_scale, "autotune": {str(k): v for k, v in choice.items()},
                   "schedule": sched, "schedule_options": sched_opts,
                   "launch": ({0: "each step launches the patches of the scenarios still running, counted on the host",
                               1: "persistent: resident workgroups walk the step's patches; running scenarios "
                                  "counted on the device"}[sched_opts.get("batch_schedule", 0)] +
                              (f"; hipGraph chunks of {sched_opts['graph_steps']} steps"
                               if sched_opts.get("graph_steps", 0) > 0 else "; eager steps"))},
        "autotune_report": {str(k): v for k, v in report.items()}, "schedule_autotune": sched_report,
        "status": status, "batch_steps_done": done, "unstable_scenarios": unstable,
        "ablated_volume_m3": {"min": float(np.nanmin(vol)), "max": float(np.nanmax(vol))},
        "T_max_K": {"min": float(np.nanmin(tmax)), "max": float(np.nanmax(tmax))},
        "scenarios": per,
    }
    print(json.dumps(out), flush=True)


def surrogate_bench(args):
    """Learned surrogate against the solver on held-out planning scenarios.

    Training data: N_TRAIN scenarios of the planning distribution (its own seed), each
    run by the batched solver with snapshots; calibration: --calib further runs; test:
    --holdout runs never seen in training.  The solver alone runs the test set in one
    batch (set-up + run + read); the surrogate predicts all of them with the ensemble
    and hands those whose disagreement estimate exceeds the threshold to the solver."""
    import torch
    from paper_2009_10400_amd import surrogate as S, workloads as W

    ds = args.duration_scale
    t_ref = 300.0 * ds
    t = time.time()
    train_sc = W.planning_scenarios(args.surrogate, seed=5, duration_scale=ds)
    if not args.shard:
        calib_sc = W.planning_scenarios(args.calib, seed=9, duration_scale=ds)
        test_sc = W.planning_scenarios(args.holdout, seed=7, duration_scale=ds)
    log(f"[surrogate] scenarios built in {time.time() - t:.1f}s")
    stream = torch.cuda.Stream(device=0)
    st = stream.cuda_stream

    t = time.time()
    if args.shard:
        k, n = (int(v) for v in args.shard.split("/"))
        lo, hi = len(train_sc) * k // n, len(train_sc) * (k + 1) // n
        snaps, t_solve = S.solve_snapshots(train_sc[lo:hi], n_snap=args.snapshots, stream=st, log=log,
                                           batch_schedule=args.surrogate_schedule,
                                           graph_steps=100 if args.surrogate_schedule else 0)
        os.makedirs(args.data_dir, exist_ok=True)
        path = os.path.join(args.data_dir, f"shard_{k:02d}_of_{n:02d}.npz")
        S.write_shard(path, train_sc, lo, snaps, per_field=args.shard_nodes)
        print(json.dumps({"shard": args.shard, "runs": hi - lo, "fields": len(snaps), "solver_seconds": t_solve,
                          "seconds": time.time() - t, "path": path, "bytes": os.path.getsize(path),
                          "duration_scale": ds}), flush=True)
        return
    shards = sorted(f for f in (os.listdir(args.data_dir) if args.data_dir else []) if f.startswith("shard_"))
    if shards:
        data = S.dataset_from_shards([os.path.join(args.data_dir, f) for f in shards], train_sc, t_ref)
        t_solve_train = None
        log(f"[surrogate] training data from {len(shards)} shards: {int(data.field.max()) + 1} fields, "
            f"{len(data.x)} samples in {time.time() - t:.1f}s")
    else:
        snaps, t_solve_train = S.solve_snapshots(train_sc, n_snap=args.snapshots, stream=st, log=log)
        data = S.make_dataset(train_sc, snaps, t_ref)
        log(f"[surrogate] training data: {len(snaps)} fields, {len(data.x)} samples in {time.time() - t:.1f}s "
            f"(solver {t_solve_train:.2f}s)")
        del snaps
    net = dict(n_freq=64, width=256, depth=5, n_out=4, sigma=args.sigma)
    ens = S.Ensemble(args.members, t_ref=t_ref, stream=st, **net)
    hist, t_train = ens.fit(data, args.epochs, batch=args.train_batch, lr=args.lr, log=log)
    log(f"[surrogate] trained {args.members} members x {args.epochs} epochs in {t_train:.1f}s")

    # MFMA roofline of the GEMM kernel: timed training steps of a separate network at the training batch size
    m0 = S.MLP(0, seed=77, stream=st, **net)
    dev = torch.device("cuda", 0)
    n = args.train_batch
    X = torch.from_numpy(data.x[:n]).to(dev)
    P = torch.from_numpy(data.p[:n]).to(dev)
    Y = torch.from_numpy(data.y[:n] / ens.y_std).to(dev)
    m0.set_timing(True)
    for _ in range(10):
        m0.train_step(X, P, Y, 1e-4)
    tm = m0.timing()
    gemm_ms, gemm_flops = tm["gemm_ms"], tm["gemm_flops"]
    m0.set_timing(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        m0.train_step(X, P, Y, 1e-4)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) / 20 * 1e3
    fwd_flops = 2.0 * sum(a * b for a, b in [(160, 256)] + [(256, 256)] * 4 + [(256, 4)])
    n_samples = len(data.x)
    m0.close()
    del data, X, P, Y

    sched = dict(batch_schedule=args.surrogate_schedule, graph_steps=100 if args.surrogate_schedule else 0)
    cal = S.solve(calib_sc, stream=st, log=log, **sched)[0]
    c = ens.calibrate(calib_sc, cal)
    log(f"[surrogate] calibration factor {c:.3g} from {len(calib_sc)} runs")

    # solver alone on the test set
    torch.cuda.synchronize()
    ref, t_solver = S.solve(test_sc, stream=st, log=log, **sched)
    rep = S.plan(ens, test_sc, threshold_K=args.threshold, stream=st, log=log, **sched)
    t_fb = rep["t_fallback"]
    t_plan = rep["t_surrogate"] + t_fb["total"]
    t_plan_gpu = rep["t_surrogate_gpu"] + t_fb["run"]
    errs, acc_err = [], []
    for k, ((kind, u, T), (ur, Tr)) in enumerate(zip(rep["results"], ref)):
        e = float(np.abs(T - Tr).max())
        errs.append(e)
        if kind == "surrogate":
            acc_err.append(e)
    # MFMA roofline of the inference kernel over the test set (HIP events around every launch)
    for m in ens.models:
        m.set_timing(True)
    ens.predict_many(test_sc)
    tms = [m.timing() for m in ens.models]
    for m in ens.models:
        m.set_timing(False)
    inf_ms = sum(t["fused_ms"] for t in tms)
    inf_flops = sum(t["fused_flops"] for t in tms)
    rise = [float((Tr - p.params["T0"]).max()) for (p, _), (_, Tr) in zip(test_sc, ref)]
    sur_only = [float(np.abs(Tm - Tr).max()) for (Tm, _, _), (_, Tr) in zip(ens.predict_many(test_sc), ref)]
    n_acc = len(acc_err)
    nt = len(test_sc)
    out = {
        "metric": "scenarios/s surrogate vs solver @0.5K", "value": nt / t_plan, "unit": "scenarios/s",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "solver_value": nt / t_solver["total"], "gain": t_solver["total"] / t_plan,
        "gpu_only": {"surrogate_value": nt / t_plan_gpu, "solver_value": nt / t_solver["run"],
                     "gain": t_solver["run"] / t_plan_gpu},
        "seconds": {"surrogate": rep["t_surrogate"], "surrogate_inference": rep["t_surrogate_gpu"],
                    "fallback_solver": t_fb, "solver_alone": t_solver, "training": t_train,
                    "training_data_solver": t_solve_train},
        "accepted": n_acc, "fallback": len(rep["rejected"]),
        "max_err_accepted_K": max(acc_err) if acc_err else None,
        "accepted_over_threshold": int(sum(e > args.threshold for e in acc_err)),
        "max_err_all_K": max(errs),
        "surrogate_only_within_threshold": float(np.mean([e <= args.threshold for e in sur_only])),
        "surrogate_only_max_err_K": float(max(sur_only)),
        "surrogate_only_median_err_K": float(np.median(sur_only)),
        "zero_rise_within_threshold": float(np.mean([r <= args.threshold for r in rise])),
        "max_rise_K": {"median": float(np.median(rise)), "max": float(max(rise))},
        "calibration_factor": c,
        "config": {"workload": f"planning scenarios (tet cubes and noisy ellipsoids, 5k-200k elements, probe 1/r^2 "
                               f"source U(20,80) W, E U(2,6) kPa, heating U(30,300) s x {ds:g}); "
                               f"{len(train_sc)} training runs x {args.snapshots} snapshots, {len(calib_sc)} "
                               f"calibration runs, {nt} held-out test runs",
                   "train_samples": n_samples, "members": args.members, "epochs": args.epochs,
                   "net": "64 Fourier frequencies + 11 parameters (160 padded) -> 5 x 256 SiLU -> 4",
                   "threshold_K": args.threshold, "duration_scale": ds, "train_batch": args.train_batch},
        "training_loss_final": [h[-1] for h in hist],
        "roofline": {"bound": "mfma", "achieved": inf_flops / (inf_ms * 1e-3) / 1e12 if inf_ms else None,
                     "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": inf_flops / (inf_ms * 1e-3) / 1e12 / 2500.0 if inf_ms else None, "traffic": None,
                     "kernel": "fused_forward_kernel (ensemble inference over the test set)",
                     "kernel_ms_total": inf_ms, "launches": args.members,
                     "flops_per_sample_forward": fwd_flops},
        "training_roofline": {"bound": "mfma", "achieved": gemm_flops / (gemm_ms * 1e-3) / 1e12, "peak": 2500.0,
                              "unit": "TFLOP/s", "frac": gemm_flops / (gemm_ms * 1e-3) / 1e12 / 2500.0,
                              "kernel": "gemm_kernel (all GEMMs of a training step)",
                              "gemm_ms_per_step": gemm_ms / 10, "train_step_ms": step_ms,
                              "samples_per_step": args.train_batch},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU domain decomposition is a design, not built).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.mlp_train_timing:
        mlp_train_timing(args)
        return
    if args.step_time_profile:
        step_time_profile(args)
        return
    if args.counters_summary:
        counters_summary(*args.counters_summary)
        return
    if args.sweep:
        sweep(args)
        return
    if args.surrogate:
        surrogate_bench(args)
        return
    import torch
    from paper_2009_10400_amd import tled, workloads as W

    t = time.time()
    p = {"ellipsoid_t4": lambda: W.ellipsoid_t4(args.elems), "cube_h8": lambda: W.cube_h8(64),
         "cube_t4": lambda: W.cube_t4()}[args.workload]()
    log(f"[bench] workload ne={p.ne} nn={p.nn} built in {time.time() - t:.1f}s")
    t = time.time()
    stream = torch.cuda.Stream(device=0)
    sim = tled.from_problem(p, device=0, stream=stream.cuda_stream, kernel_variant=args.variant,
                            graph_steps=args.graph_steps, patch_elems=args.patch_elems,
                            block_size=args.block_size, reorder=args.reorder, shared_update=args.shared_update,
                            finalize=False)
    if args.thermal_dose:
        sim.set_thermal_dose(7.39e39, 2.577e5)
    sim.finalize()
    info = sim.info()
    log(f"[bench] finalize {time.time() - t:.1f}s info={info}")
    # capture the hipGraphs the timed step(K) calls replay (set-up only: nothing runs) before the
    # warm-up steps, so that no capture leaves the GPU idle between them and the timed regions (an
    # idle GPU lowers its clock: `--step-time-profile` measures what idling costs a short region)
    sim.prepare(args.steps)
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    # --repeats timed regions of exactly K steps each, every one bracketed by device
    # synchronisation; the line reports their median (all of them under "repeats")
    reps = []
    for _ in range(max(1, args.repeats)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim.step(args.steps)
        torch.cuda.synchronize()
        reps.append(1e3 * (time.perf_counter() - t1) / args.steps)
    sim.sync()
    ms_per_step = float(np.median(reps))
    value = p.ne / (ms_per_step * 1e-3)
    log(f"[bench] {len(reps)} timed regions of {args.steps} steps (ms/step): {[round(r, 5) for r in reps]}, "
        f"median {ms_per_step:.5f} -> {value:.4g} element-updates/s")
    # context for short regions: the first few hundred steps of a run cost more per step, and
    # each region carries its own launch and synchronisation; one more region of at least 2000
    # steps gives the per-step time a long run approaches
    steady = None
    if args.steps < 2000:
        n_long = 2000
        sim.prepare(n_long)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim.step(n_long)
        torch.cuda.synchronize()
        ms_long = 1e3 * (time.perf_counter() - t1) / n_long
        steady = {"steps": n_long, "ms_per_step": ms_long, "value": p.ne / (ms_long * 1e-3),
                  "note": "one further timed region of this many steps, same bracketing; context only"}
        log(f"[bench] one region of {n_long} steps: {ms_long:.5f} ms/step")

    # dominant kernel, timed with HIP events on the library's stream
    kt = sim.kernel_times(args.kernel_steps)
    sim.sync()
    kname = "patch_kernel" if info["kernel_variant"] >= 2 else ("t4_element_kernel" if p.npe == 4 else "h8_element_kernel")
    eb = elem_bytes(p.npe, info["n_prony"])
    fused = info["shared_update"] == 1
    chunk = args.graph_steps if args.graph_steps > 0 else (50 if args.graph_steps == 0 else 100)

    def n_chunks(k):   # tled_step(k) and tled_kernel_times(k) run ceil(k / chunk) chunks
        return -(-k // chunk)

    if info["kernel_variant"] >= 2:
        n_interior = info["n_nodes"] - info["n_shared_nodes"]
        # per launch, averaged over the timed steps: a fused launch also advances the shared
        # nodes by the previous step; the first launch of each chunk does not
        f_frac = (args.kernel_steps - n_chunks(args.kernel_steps)) / args.kernel_steps if fused else 0.0
        alg_bytes = eb * p.ne + NODE_BYTES * (n_interior + f_frac * info["n_shared_nodes"])
    else:
        alg_bytes = eb * p.ne + 16.0 * p.npe * p.ne   # plus the nodal outputs it writes
    achieved = alg_bytes / (kt["element_ms"] * 1e-3) / 1e9
    key = workload_key(p.name, args.elems)
    traffic = traffic_from_profiles(kname, key, info)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
            "kernel_ms": kt["element_ms"], "second_kernel_ms": kt["node_ms"],
            "algorithmic_bytes_per_launch": alg_bytes}
    log(f"[bench] kernel times {kt}")
    # the whole step's HBM traffic (both kernels, counted) against peak and against a plain copy
    step_hbm = None
    rec = traffic_record(key, info) if info["kernel_variant"] >= 2 else None
    if rec is not None:
        sf, sw = rec["shared_node_kernel_kib"]
        shared_bytes = 1024.0 * (sf * rec["fetch_scale"] + sw * rec["write_scale"])
        if fused:
            # per timed step: the fused patch kernel, except the unfused first launch of each
            # chunk, and one shared-node kernel per chunk
            nc = n_chunks(args.steps)
            first = rec.get("chunk_first_patch_kernel_kib")
            first_bytes = (1024.0 * (first[0] * rec["fetch_scale"] + first[1] * rec["write_scale"])
                           if first else rec["bytes_per_launch"])
            step_bytes = ((args.steps - nc) * rec["bytes_per_launch"] + nc * (first_bytes + shared_bytes)) / args.steps
        else:
            step_bytes = rec["bytes_per_launch"] + shared_bytes
        gbs = step_bytes / (ms_per_step * 1e-3) / 1e9
        cbw = copy_bandwidth()
        step_hbm = {"bytes_counted": step_bytes, "GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
                    "copy_GBs": cbw, "frac_of_copy": gbs / cbw,
                    "note": "counted FETCH+WRITE bytes of the patch and shared-node kernels per step / "
                            "whole-step time; copy = 1 GiB device copy on the same GPU"}
        log(f"[bench] step HBM {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.3f} of peak, {gbs / cbw:.3f} of copy {cbw:.0f} GB/s)")
    out = {
        "metric": "coupled element-updates/s (HBM % peak)",
        "value": value, "unit": "element-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": {
                       "ellipsoid_t4": f"noisy ellipsoid 0.2x0.15x0.1 m, {p.ne} T4 / {p.nn} nodes, 2 Prony terms, "
                                       f"shrinkage above 323 K, 20 mm 1/r^4 line source (10 W), random numbering",
                       "cube_h8": f"0.1 m cube, {p.ne} H8 (64^3, one-point + hourglass) / {p.nn} nodes, "
                                  f"fibre field, mu(T), 1/r^2 point source (10 W)",
                       "cube_t4": f"0.04 m cube, {p.ne} T4 / {p.nn} nodes, 1 Prony term, Gaussian source "
                                  f"(5e7 W/m^3, sigma 4 mm)"}[args.workload],
                   "n_elems": p.ne, "n_nodes": p.nn, "kernel_variant": info["kernel_variant"],
                   "graph_steps": args.graph_steps or 50, "patches": info["n_patches"],
                   "shared_nodes": info["n_shared_nodes"],
                   "shared_node_fraction": info["n_shared_nodes"] / max(1, info["n_nodes"]),
                   "patch_lds_bytes": info["patch_lds_bytes"],
                   "patch_wgs_per_cu": info["patch_wgs_per_cu"],
                   "shared_update": {1: "fused into the next step's patch kernel",
                                     2: "shared-node kernel every step"}.get(info["shared_update"], "none"),
                   "patch_order": {-1: "as generated", 2: "Morton runs"}.get(args.reorder, "coordinate bisection"),
                   "dt": sim.dt},
        "roofline": roof,
        "step_hbm": step_hbm,
        "repeats": {"ms_per_step": reps, "median_ms_per_step": ms_per_step,
                    "note": "value and ms_per_step are the median of these timed regions of K steps each"},
        "long_region": steady,
        "thermal_dose": None if not args.thermal_dose else dose_summary(sim),
    }
    if not args.no_cpu_baseline and p.npe == 4:
        steps = args.cpu_steps or max(3, int(100e6 / p.ne))
        log(f"[bench] CPU baseline: oracle {steps} steps")
        out["cpu_baseline"] = cpu_baseline(p, sim.dt, steps)
        nt = host_threads()
        if nt > 1:
            log(f"[bench] CPU baseline on {nt} host cores")
            out["cpu_all_cores"] = cpu_baseline_all_cores(p, sim.dt, max(3, steps // 2), nt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
