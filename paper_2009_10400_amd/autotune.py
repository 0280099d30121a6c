"""Autotuner of the batched planning sweep: patch size per mesh-size bucket.

The fused kernels process one patch of consecutive elements per workgroup.  The
best patch size depends on the mesh: it trades the number of nodes shared
between patches (assembled by a second kernel) against the number of
workgroups that can fill the GPU and the idle tail of the last round.  For each
size bucket the tuner builds a small batch of that bucket's scenarios, times a
few steps of it per candidate patch size (HIP events on the library's stream)
and keeps the fastest.  Timing only: the physics does not depend on the choice.
"""
from __future__ import annotations

import time

import numpy as np

BUCKETS = ((0, 15_000), (15_000, 50_000), (50_000, 10**9))
CANDIDATES = (192, 256, 320, 384, 448, 504)


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
