"""Long GPU-only runs at the workloads' stated lengths (no oracle: its serial FP64 steps would
take hours here): the 64^3 H8 cube through its 60 s of heating and 30 s of cooling (319 206
steps), and the 1.0M-tet ellipsoid through its 20 000 steps.  Each runs twice from scratch and
must give the same bits; no device flag may be raised, every field stays finite, the heat held
never exceeds the heat deposited (perfusion and adiabatic walls only remove or keep it), the
temperature peak rises while the source is on and falls once it is off."""
import numpy as np
import pytest

from harness import gpu_sim, log
from paper_2009_10400_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(p, segments):
    """Steps the segments in order; returns the fields and the monitors after each segment."""
    sim = gpu_sim(p)                     # the library's default kernel variant
    mons = []
    for n in segments:
        sim.step(n)
        sim.sync()
        mons.append(sim.monitors())
    return sim, sim.read_u(), sim.read_T(), mons


def _heat_bounds(sim, p, T, t_heat):
    """Heat content above T0 (sum of C_a (T_a - T0)) and the energy the source deposited."""
    lum = sim.lumped()
    held = float((lum["C"] * (T - p.params["T0"])).sum())
    deposited = float(lum["Qr"].sum()) * t_heat
    return held, deposited


def test_cube_h8_64_heating_and_cooling_90s():
    p = W.cube_h8(n=64)                  # 10 W point source on for 60 s
    sim0 = gpu_sim(p)
    dt = sim0.dt
    sim0.close()
    n_heat = int(round(60.0 / dt))
    n_total = int(round(90.0 / dt))
    log(f"  H8 64^3: dt={dt:.6e} s, {n_heat} heating + {n_total - n_heat} cooling steps")
    results = []
    for rep in range(2):
        sim, u, T, mons = _run(p, [n_heat, n_total - n_heat])
        results.append((u, T))
        log(f"  run {rep}: monitors at 60 s {mons[0]}, at 90 s {mons[1]}")
        for m in mons:
            assert m["flags"] == 0
        assert np.isfinite(u).all() and np.isfinite(T).all()
        assert mons[0]["T_max"] > p.params["T0"] + 1.0          # the probe region heated up
        assert mons[1]["T_max"] < mons[0]["T_max"]               # and cools once the source is off
        held, deposited = _heat_bounds(sim, p, T, 60.0)
        log(f"  heat held {held:.1f} J of {deposited:.1f} J deposited")
        assert 0.0 < held <= deposited
        sim.close()
    assert np.array_equal(results[0][0], results[1][0]) and np.array_equal(results[0][1], results[1][1])


def test_ellipsoid_t4_1m_20000_steps():
    p = W.ellipsoid_t4(1_000_000)        # 10 W line source on throughout
    results = []
    for rep in range(2):
        sim, u, T, mons = _run(p, [10000, 10000])
        results.append((u, T))
        log(f"  run {rep}: monitors at 10000 {mons[0]}, at 20000 {mons[1]}")
        for m in mons:
            assert m["flags"] == 0
        assert np.isfinite(u).all() and np.isfinite(T).all()
        assert mons[1]["T_max"] > mons[0]["T_max"] > p.params["T0"]
        held, deposited = _heat_bounds(sim, p, T, 20000 * sim.dt)
        log(f"  heat held {held:.2f} J of {deposited:.2f} J deposited")
        assert 0.0 < held <= deposited
        sim.close()
    assert np.array_equal(results[0][0], results[1][0]) and np.array_equal(results[0][1], results[1][1])
