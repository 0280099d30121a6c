"""Nodes shared between patches advanced inside the next step's patch kernel
(``shared_update = 1``, the default for single problems) against a shared-node kernel
after every step (``shared_update = 2``): the same bits in every field and monitor, for
graph chunks, eager chunks and calls of one step (where nothing is fused)."""
import numpy as np
import pytest

from harness import gpu_sim, log
from paper_2009_10400_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ellipsoid():
    p = W.ellipsoid_t4(30000)
    p.params = dict(p.params, shrink_T=p.params["T0"] + 0.3, shrink_width=1.0)
    return p


def _cube_t4_laws():
    # four Prony terms, mu(T), c(T)/k(T), metabolic heat and arterial temperature
    p = W.cube_t4()
    p.params = dict(p.params, g=[0.2, 0.2, 0.1, 0.1], tau=[0.05, 0.2, 1.0, 5.0], n_prony=4,
                    muT_on=1, muT_lo=310.15, muT_hi=311.0, ckT_on=1, ckT_lo=310.15, ckT_hi=312.0,
                    Q_met=3e4, T_art=311.0)
    return p


def _cube_t4_no_prony_fixed_T():
    p = W.cube_t4()
    p.params = dict(p.params, eta=0.0, g=[], tau=[], n_prony=0)
    fix = np.zeros(p.nn, dtype=np.uint8) if p.fix is None else p.fix.copy()
    top = p.X[:, 2] >= p.X[:, 2].max() - 1e-12
    fix[top] |= 8
    p.fix = fix
    p.Tfix = np.full(p.nn, p.params["T0"] + 2.0)
    return p


CASES = {
    "ellipsoid_t4_30k": _ellipsoid,
    "cube_h8_12": lambda: W.cube_h8(n=12),
    "cube_t4_laws": _cube_t4_laws,
    "cube_t4_no_prony_fixed_T": _cube_t4_no_prony_fixed_T,
}
CHUNKS = [1, 2, 123, 3, 1, 50]      # tled_step calls: lengths 1 (no fusion), 2, remainders


def _run(p, shared_update, graph_steps):
    sim = gpu_sim(p, kernel_variant=2, shared_update=shared_update, graph_steps=graph_steps)
    assert sim.info()["shared_update"] == shared_update
    mons = []
    for c in CHUNKS:
        sim.step(c)
        mons.append(sim.monitors())
    sim.sync()
    st = sim.read_state()
    sim.close()
    return st, mons


@pytest.mark.parametrize("graph_steps", [50, 7, -1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_fused_shared_nodes_bitwise(name, graph_steps):
    p = CASES[name]()
    log(f"  {name} ne={p.ne} graph_steps={graph_steps}")
    ref, mref = _run(p, 2, graph_steps)
    got, mgot = _run(p, 1, graph_steps)
    assert ref["step"] == got["step"] == sum(CHUNKS)
    for k in ("u", "v", "T", "theta"):
        a, b = np.asarray(ref[k]), np.asarray(got[k])
        assert a.shape == b.shape
        diff = np.flatnonzero(a.view(np.uint8) != b.view(np.uint8)) if a.size else []
        assert len(diff) == 0, f"{k}: {len(diff)} bytes differ, max |diff| {np.abs(a - b).max()}"
    assert np.abs(ref["u"]).max() > 1e-9
    for m1, m2 in zip(mref, mgot):
        assert m1 == m2
