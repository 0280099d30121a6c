"""Autotuner of the batched planning sweep: patch size per mesh-size bucket, then the batch's
launch schedule.

The fused kernels process one patch of consecutive elements per workgroup.  The
best patch size depends on the mesh: it trades the number of nodes shared
between patches (assembled by a second kernel) against the number of
workgroups that can fill the GPU and the idle tail of the last round.  For each
size bucket the tuner builds a small batch of that bucket's scenarios, times a
few steps of it per candidate patch size (HIP events on the library's stream)
and keeps the fastest.  The schedule (how each batch step is launched: eager steps or hipGraph
chunks over the scenarios the host counts as running, or the persistent kernels in graph chunks of
a given length) is a property of the whole batch: the tuner runs a sample of the batch's scenarios, with
their uneven end steps scaled down, to completion under each candidate and keeps the fastest.
Timing only: the physics does not depend on either choice (a scenario's fields are the same bits
under every schedule).
"""
from __future__ import annotations

import time

import numpy as np

BUCKETS = ((0, 15_000), (15_000, 50_000), (50_000, 10**9))
CANDIDATES = (192, 256, 320, 384, 448, 504)
SCHEDULES = {
    "prefix-eager": dict(batch_schedule=0, graph_steps=-1),
    "prefix-graph-50": dict(batch_schedule=0, graph_steps=50),
    "persistent-graph-100": dict(batch_schedule=1, graph_steps=100),
    "persistent-graph-400": dict(batch_schedule=1, graph_steps=400),
}


def bucket_of(n_elems: int) -> int:
    for b, (lo, hi) in enumerate(BUCKETS):
        if lo <= n_elems < hi:
            return b
    return len(BUCKETS) - 1


def tune(scenarios, device: int = 0, steps: int = 60, sample: int = 6, candidates=CANDIDATES,
         stream=None, log=print):
    """scenarios: list of Problems (time step: their cfl fraction of the critical step).
    Returns ({bucket: patch_elems}, report)."""
    from . import tled
    choice, report = {}, {}
    for b in range(len(BUCKETS)):
        idx = [k for k, p in enumerate(scenarios) if bucket_of(p.ne) == b][:sample]
        if not idx:
            continue
        best, times = None, {}
        for pe in candidates:
            bt = tled.Batch(device, stream=stream)
            bt.set_options(graph_steps=-1)
            for k in idx:
                bt.add(scenarios[k], cfl=scenarios[k].cfl, t_end=1e6, patch_elems=pe)
            bt.finalize()
            bt.step(10)                                   # warm-up
            kt = bt.kernel_times(steps)
            per_step = kt["element_ms"] + kt["node_ms"]
            ne = sum(scenarios[k].ne for k in idx)
            times[pe] = per_step
            rate = ne / (per_step * 1e-3)
            log(f"[autotune] bucket {b} ({len(idx)} scenarios, {ne} elements) patch {pe}: "
                f"{per_step * 1e3:.2f} us/step, {rate:.3g} element-updates/s")
            bt.close()
            if best is None or per_step < times[best]:
                best = pe
        choice[b] = best
        report[b] = {"scenarios": len(idx), "ms_per_step": times, "best": best}
    return choice, report


def tune_schedule(scenarios, durations, patch_choice, device: int = 0, sample: int = 32, batch_steps: int = 3000,
                  schedules=None, stream=None, log=print):
    """scenarios, durations: the batch (Problems and heating times).  A sample of `sample`
    scenarios spread over the batch keeps the ratios of their step counts, scaled so that the
    longest runs `batch_steps` steps; it runs to completion once per schedule, timed from after
    finalize and tled_prepare_steps (graph capture that the full batch would amortise over many
    more steps).  Returns (name, options, report)."""
    import torch
    from . import tled
    schedules = schedules or SCHEDULES
    n = len(scenarios)
    idx = sorted(set(np.linspace(0, n - 1, min(sample, n)).round().astype(int).tolist()))
    # a scenario's step count is its duration over its time step (cfl x its critical step)
    dts = []
    for k in idx:
        s = tled.from_problem(scenarios[k], device=-1, finalize=False)
        dts.append(scenarios[k].cfl * s.critical_dt())
        s.close()
    ends = [durations[k] / dt for k, dt in zip(idx, dts)]
    scale = batch_steps / max(ends)
    steps = [max(1, int(round(e * scale))) for e in ends]
    report, best = {}, None
    for name, opts in schedules.items():
        bt = tled.Batch(device, stream=stream)
        bt.set_options(**opts)
        for k, dt, nk in zip(idx, dts, steps):
            bt.add(scenarios[k], dt=dt, n_steps=nk, patch_elems=patch_choice.get(bucket_of(scenarios[k].ne), 0))
        bt.finalize()
        bt.prepare(max(steps))
        bt.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.run()
        bt.sync()
        sec = time.perf_counter() - t0
        bt.close()
        report[name] = sec
        log(f"[autotune] schedule {name}: {sec * 1e3:.1f} ms for {len(idx)} scenarios, {max(steps)} batch steps")
        if best is None or sec < report[best]:
            best = name
    return best, dict(schedules[best]), {"sample": len(idx), "batch_steps": max(steps), "seconds": report}
