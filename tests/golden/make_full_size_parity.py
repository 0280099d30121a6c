"""Writes the expected values of the full-size 1000-step parity tests.

For each full-size workload the FP64 oracle advances 1000 steps from the initial
state at 0.8 of the oracle's own critical step.  Stored per workload
(``full_size_<name>.npz``, loadable with ``allow_pickle=False``):

* ``dt``, ``steps`` and ``fingerprint`` (SHA-256 of the generated inputs, so a
  change of the generator is detected instead of compared against stale values);
* whole-field figures of the oracle's final state: ``u_max`` (max |u| over all
  components), ``T_max``, ``T_min`` and ``heat`` (sum of lumped volume x T);
* the displacement and temperature of a seeded sample of 4096 nodes plus the
  64 nodes of largest |u| and the 64 of largest T.

Only the oracle and the seeded input generators are called.  Run from the
repository root:  ``python tests/golden/make_full_size_parity.py [name ...]``
(about 3 minutes for the ellipsoid and 2 for the cube on one core each; the
two run in parallel processes).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time
from multiprocessing import Process

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

STEPS = 1000
N_SAMPLE = 4096
N_EXTREME = 64


def problems():
    """The full-size workloads of the parity bar (the same constructions the tests use)."""
    from paper_2009_10400_amd import workloads as W

    def ellipsoid():
        p = W.ellipsoid_t4(1_000_000)
        # shrinkage ramp moved down to where the first 1000 steps' heating reaches it
        p.params = dict(p.params, shrink_T=p.params["T0"] + 0.05, shrink_width=0.5)
        return p

    return {"ellipsoid_t4_1m": ellipsoid, "cube_h8_64": lambda: W.cube_h8(n=64)}


def fingerprint(p) -> str:
    h = hashlib.sha256()
    for a in (p.X, p.conn, p.a0, p.q, p.fix):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    h.update(repr(sorted((k, v) for k, v in p.params.items())).encode())
    h.update(repr((p.npe, p.t_on, p.t_off, p.gamma, p.cfl)).encode())
    return h.hexdigest()


def sample_nodes(nn: int, u, T):
    rng = np.random.default_rng(12345)
    pick = set(rng.choice(nn, size=min(N_SAMPLE, nn), replace=False).tolist())
    pick |= set(np.argsort(-np.abs(u).max(1))[:N_EXTREME].tolist())
    pick |= set(np.argsort(-T)[:N_EXTREME].tolist())
    return np.array(sorted(pick), dtype=np.int64)


def make(name: str):
    import oracle

    t = time.time()
    p = problems()[name]()
    o = oracle.OracleSim(p.npe, p.X, p.conn, p.params, a0=p.a0, q=p.q, fix=p.fix, Tfix=p.Tfix,
                         t_on=p.t_on, t_off=p.t_off, dt=0.0, gamma=p.gamma)
    dt = p.cfl * o.critical_dt
    o = oracle.OracleSim(p.npe, p.X, p.conn, p.params, a0=p.a0, q=p.q, fix=p.fix, Tfix=p.Tfix,
                         t_on=p.t_on, t_off=p.t_off, dt=dt, gamma=p.gamma)
    st = o.initial_state(p.params["T0"])
    print(f"[{name}] ne={p.ne} nn={p.nn} dt={dt:.6e} set-up {time.time() - t:.1f}s", flush=True)
    for k in range(10):
        o.run(st, STEPS // 10)
        print(f"[{name}] {(k + 1) * STEPS // 10} steps, {time.time() - t:.1f}s", flush=True)
    u, T = st["u"], st["T"]
    nodes = sample_nodes(p.nn, u, T)
    Vl = o.lumped()["Vl"]
    out = os.path.join(HERE, f"full_size_{name}.npz")
    np.savez_compressed(out, dt=dt, steps=STEPS, fingerprint=np.array(fingerprint(p)),
                        u_max=np.abs(u).max(), T_max=T.max(), T_min=T.min(), heat=float((Vl * T).sum()),
                        nodes=nodes, u=u[nodes], T=T[nodes])
    print(f"[{name}] wrote {out}: u_max {np.abs(u).max():.4e} m, T_max {T.max():.4f} K", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(problems())
    procs = [Process(target=make, args=(n,)) for n in names]
    for pr in procs:
        pr.start()
    for pr in procs:
        pr.join()
    sys.exit(max(abs(pr.exitcode or 0) for pr in procs))
