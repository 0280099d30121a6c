"""Full-size parity after 1000 steps in the benchmark's launch configuration (fused patch
kernels in the library's default variant, hipGraph chunks of 50 steps): the ~1.0M-tet ellipsoid (two Prony terms, shrinkage
with its ramp moved down so that it engages, fibre field, 1/r^4 line source) and the 64^3 H8
cube (hourglass control, mu(T), fibre field, 1/r^2 source), against the FP64 oracle's
1000-step states stored by ``tests/golden/make_full_size_parity.py``.

Bar: max-abs displacement error over the stored nodes (a seeded sample of 4096 plus the 64
of largest |u| and the 64 hottest) relative to the oracle's max |u| over all nodes <= 1e-4,
max-abs temperature error <= 0.01 K; the GPU's whole-field max |u|, T max / min and heat
content agree with the oracle's to the same bar.
"""
import os
import sys

import numpy as np
import pytest

from harness import T_ABS_TOL, U_REL_TOL, gpu_sim, log

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_full_size_parity as G  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["ellipsoid_t4_1m", "cube_h8_64"])
def test_full_size_1000_steps(name):
    ref = np.load(os.path.join(HERE, "golden", f"full_size_{name}.npz"), allow_pickle=False)
    p = G.problems()[name]()
    assert str(ref["fingerprint"]) == G.fingerprint(p), \
        "generated inputs changed: run tests/golden/make_full_size_parity.py again"
    steps = int(ref["steps"])
    log(f"  {name}: ne={p.ne} nn={p.nn} dt={float(ref['dt']):.6e} steps={steps}")
    sim = gpu_sim(p, dt=float(ref["dt"]))          # the library's default variant, as benchmarked
    log(f"  {name}: kernel variant {sim.info()['kernel_variant']}")
    sim.step(steps)
    sim.sync()
    u, T = sim.read_u(), sim.read_T()
    nodes = ref["nodes"]
    u_max = float(ref["u_max"])
    u_rel = float(np.abs(u[nodes] - ref["u"]).max() / u_max)
    T_abs = float(np.abs(T[nodes] - ref["T"]).max())
    Vl = sim.lumped()["Vl"]
    heat_err = abs(float((Vl * T).sum()) - float(ref["heat"])) / Vl.sum()
    whole = {"u_max_rel": abs(np.abs(u).max() - u_max) / u_max, "T_max": abs(T.max() - float(ref["T_max"])),
             "T_min": abs(T.min() - float(ref["T_min"])), "heat_per_volume_K": heat_err}
    log(f"  {name}: sampled {len(nodes)} nodes u_rel={u_rel:.3e} T_abs={T_abs:.3e} K, whole field {whole}, "
        f"oracle u_max={u_max:.4e} m T_max={float(ref['T_max']):.4f} K")
    assert sim.monitors()["step"] == steps
    assert u_rel <= U_REL_TOL and T_abs <= T_ABS_TOL
    assert whole["u_max_rel"] <= U_REL_TOL
    assert whole["T_max"] <= T_ABS_TOL and whole["T_min"] <= T_ABS_TOL and heat_err <= T_ABS_TOL
    assert u_max > 1e-9 and float(ref["T_max"]) - p.params["T0"] > 0.05      # not a trivial field
