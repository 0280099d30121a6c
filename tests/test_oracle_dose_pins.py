"""Pins of the oracle's thermal dose: CEM43 (Sapareto and Dewey) and the Arrhenius damage
integral (Henriques and Moritz), the thermal-damage measures Section 7 names beside an isotherm.

CEM43 counts equivalent minutes at 43 C at a rate R^(43 - T_C) per minute, R = 0.5 at and above
43 C and 0.25 below: every kelvin above 43 C doubles the rate, every kelvin below quarters it.
The Arrhenius integral grows at A exp(-Ea / (R_gas T)) per second with T in kelvin.  The expected
values below follow from those definitions by hand (powers of two, and Arrhenius parameters whose
exponent cancels at a chosen temperature), not by evaluating the formulas again."""
import math

import numpy as np
import pytest

import oracle
from paper_2009_10400_amd import workloads as W

R_GAS = 8.314462618
T43 = 316.15


def _dose(T, dt, n, A=0.0, Ea=0.0):
    T = np.asarray(T, dtype=float)
    c, o = np.zeros(T.size), np.zeros(T.size)
    for _ in range(n):
        oracle.thermal_dose(T, dt, A, Ea, c, o)
    return c, o


def test_cem43_at_43C_counts_minutes():
    """240 minutes at 43 C are 240 equivalent minutes (the usual necrosis threshold)."""
    c, _ = _dose([T43], 60.0, 240)
    assert c[0] == pytest.approx(240.0, rel=1e-12)


@pytest.mark.parametrize("dK,rate", [(1, 2.0), (3, 8.0), (7, 128.0), (-1, 0.25), (-2, 1.0 / 16), (-5, 1.0 / 1024)])
def test_cem43_doubles_per_kelvin_above_and_quarters_below(dK, rate):
    c, _ = _dose([T43 + dK], 30.0, 4)          # two minutes
    assert c[0] == pytest.approx(2.0 * rate, rel=1e-12)


def test_cem43_continuous_at_43C():
    for T in (T43 - 1e-9, T43, T43 + 1e-9):
        c, _ = _dose([T], 60.0, 1)
        assert c[0] == pytest.approx(1.0, rel=1e-8)


def test_arrhenius_rate_set_to_one_per_second():
    """A = e^100 /s and Ea = 100 R_gas (300 K): the exponent cancels at 300 K (rate 1 /s); at
    600 K it is 100 - 50, rate e^50 /s; at 150 K, 100 - 200, rate e^-100 /s."""
    A, Ea = math.exp(100.0), 100.0 * R_GAS * 300.0
    _, o = _dose([300.0], 0.5, 10, A, Ea)
    assert o[0] == pytest.approx(5.0, rel=1e-12)
    _, o = _dose([600.0], 1e-3, 3, A, Ea)
    assert o[0] == pytest.approx(3e-3 * math.exp(50.0), rel=1e-12)
    _, o = _dose([150.0], 2.0, 1, A, Ea)
    assert o[0] == pytest.approx(2.0 * math.exp(-100.0), rel=1e-12)


def test_arrhenius_off_without_frequency_factor():
    c, o = _dose([350.0], 1.0, 5, 0.0, 1e5)
    assert o[0] == 0.0 and c[0] > 0.0


def test_dose_over_a_time_loop_at_held_temperatures():
    """In the time loop the dose is added at the temperature each step ends at: nodes held at
    45 C accumulate dt/60 x 4 per step, a free body at a uniform 43 C with no source and
    perfusion at 43 C stays there and accumulates dt/60 per step."""
    p = W.cube_t4(n=2, L=0.01)
    params = dict(p.params, T0=T43, T_art=T43)
    fix = np.zeros(p.nn, dtype=np.uint8)
    fix[:3] = 8
    Tfix = np.full(p.nn, T43 + 2.0)
    dt = 1e-3
    o = oracle.OracleSim(p.npe, p.X, p.conn, params, a0=p.a0, q=None, fix=fix, Tfix=Tfix, dt=dt, gamma=p.gamma)
    st = o.initial_state(T43)
    st["T"][:3] = T43 + 2.0
    o.run_with_dose(st, 7, 0.0, 0.0)
    assert np.allclose(st["cem43"][:3], 7 * dt / 60.0 * 4.0, rtol=1e-12)
    free = np.arange(3, p.nn)
    # the held nodes warm their neighbours slightly; the far corner stays at 43 C to rounding
    far = free[np.argmax(np.linalg.norm(p.X[free] - p.X[:3].mean(0), axis=1))]
    assert st["cem43"][far] == pytest.approx(7 * dt / 60.0, rel=1e-6)
