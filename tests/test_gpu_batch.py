"""Batched planning sweep on the GPU: many scenarios advanced together by the fused kernels.

Each scenario of a batch must give bit for bit what the same scenario gives when run on its own
(same patch size), hold its state after its own step count, and agree with the FP64 oracle."""
import numpy as np
import pytest

from harness import T_ABS_TOL, U_REL_TOL, errors, log, oracle_sim
from paper_2009_10400_amd import workloads as W

pytestmark = pytest.mark.gpu


def small_batch():
    sc = W.planning_scenarios(6, seed=11, lo=1500, hi=9000, duration_scale=1.0)
    steps = [150, 310, 90, 240, 200, 275]
    return sc, steps


def critical_dt(problem):
    from paper_2009_10400_amd import tled
    s = tled.from_problem(problem, device=-1, finalize=False)
    dt = s.critical_dt()
    s.close()
    return dt


@pytest.mark.parametrize("graph_steps,schedule", [(40, 0), (-1, 0), (40, 1), (-1, 1), (7, 1)])
def test_batch_equals_single_runs_bitwise_and_holds(graph_steps, schedule):
    # scenarios end at different steps, most of them inside a chunk: a step launches only the
    # scenarios still running (graph chunks: those running at the chunk's first step); the
    # persistent schedule (1) counts them on the device and the resident workgroups walk their patches
    from paper_2009_10400_amd import tled
    sc, steps = small_batch()
    b = tled.Batch(0)
    b.set_options(graph_steps=graph_steps, batch_schedule=schedule)
    dts = []
    for (p, _), n in zip(sc, steps):
        dt = 0.8 * critical_dt(p)
        dts.append(dt)
        b.add(p, dt, n)
    b.finalize()
    b.run()
    b.sync()
    info = b.batch_info()
    log("  batch", info)
    assert info["step"] == max(steps)
    for k, ((p, _), n) in enumerate(zip(sc, steps)):
        ub, Tb = b.read(k)
        # same patches as the batch's default (T4 448, H8 256): same bits
        s = tled.from_problem(p, dt=dts[k], device=0, kernel_variant=2, graph_steps=40,
                              patch_elems=448 if p.npe == 4 else 256)
        s.step(n)
        us, Ts = s.read_u(), s.read_T()
        assert np.array_equal(ub, us), (k, float(np.abs(ub - us).max()), float(np.abs(us).max()))
        assert np.array_equal(Tb, Ts), (k, float(np.abs(Tb - Ts).max()))
        assert Tb.max() > p.params["T0"]
    # stepping further changes nothing: every scenario has reached its end
    before = [b.read(k) for k in range(len(sc))]
    b.step(25)
    for k in range(len(sc)):
        u2, T2 = b.read(k)
        assert np.array_equal(before[k][0], u2) and np.array_equal(before[k][1], T2)
    # the bulk read returns the same fields, scenario by scenario
    for k, (ua, Ta) in enumerate(b.read_all()):
        assert np.array_equal(before[k][0], ua) and np.array_equal(before[k][1], Ta)


def test_batch_scenarios_against_oracle_and_monitors():
    from paper_2009_10400_amd import tled
    sc, steps = small_batch()
    sc, steps = sc[:3], steps[:3]
    b = tled.Batch(0)
    dts = []
    for (p, _), n in zip(sc, steps):
        dt = 0.8 * critical_dt(p)
        dts.append(dt)
        b.add(p, dt, n)
    b.finalize()
    b.run()
    thr = W.T_BODY + 0.05
    tmax, vol = b.scenario_monitors(thr)
    for k, ((p, _), n) in enumerate(zip(sc, steps)):
        u, T = b.read(k)
        o = oracle_sim(p, dts[k])
        st = o.initial_state(p.params["T0"])
        o.run(st, n)
        err = errors(st["u"], u, st["T"], T)
        log(f"  scenario {k} ({p.meta['kind']}, ne={p.ne}, E={p.meta['E']:.0f}, P={p.meta['power']:.1f} W)", err)
        assert err["u_rel"] <= U_REL_TOL and err["T_abs"] <= T_ABS_TOL
        assert tmax[k] == pytest.approx(T.max(), abs=1e-4)
        Vl = o.lumped()["Vl"]
        hot = T >= thr
        assert vol[k] == pytest.approx(Vl[hot].sum(), rel=1e-5, abs=1e-15)


def test_batch_fields_independent_of_host_threads_and_duration_api(monkeypatch):
    """A batch set up on 1 or 4 host threads, with time steps chosen at finalize, runs to the
    same bits; the chosen steps equal the explicit ones."""
    from paper_2009_10400_amd import tled
    sc = W.planning_scenarios(5, seed=13, lo=1500, hi=9000, duration_scale=2e-4)
    outs = []
    for threads in ("1", "4"):
        monkeypatch.setenv("TLED_HOST_THREADS", threads)
        b = tled.Batch(0)
        b.set_options(graph_steps=30)
        for p, dur in sc:
            b.add(p, cfl=0.8, t_end=dur)
        b.finalize()
        steps = [b.scenario_steps(k) for k in range(len(sc))]
        log(f"  threads {threads}: steps {[n for _, n in steps]}")
        b.run()
        outs.append((steps, b.read_all()))
        b.close()
    (s1, f1), (s4, f4) = outs
    assert s1 == s4
    for (u1, T1), (u4, T4) in zip(f1, f4):
        assert np.array_equal(u1, u4) and np.array_equal(T1, T4)
    # explicit dt / n_steps give the same run
    b = tled.Batch(0)
    b.set_options(graph_steps=30)
    for (p, _), (dt, n) in zip(sc, s1):
        b.add(p, dt, n)
    b.finalize()
    b.run()
    for (u1, T1), (u, T) in zip(f1, b.read_all()):
        assert np.array_equal(u1, u) and np.array_equal(T1, T)


@pytest.mark.parametrize("variant,schedule", [(2, 0), (3, 0), (3, 1)])
def test_h8_batch_equals_single_runs_bitwise(variant, schedule):
    """H8 scenarios of different sizes and materials in one batch: each equal bit for bit to its own
    run with the same patch size and kernel variant, and held after its step count (eager prefix
    launches, or the persistent kernels)."""
    from paper_2009_10400_amd import tled
    probs = [W.cube_h8(n=n, L=0.02 * n / 6, power=p) for n, p in ((6, 2.0), (9, 5.0), (7, 3.0))]
    probs[1].params = dict(probs[1].params, mu=1500.0, eta=3000.0)
    steps = [120, 200, 60]
    b = tled.Batch(0)
    b.set_options(graph_steps=40, kernel_variant=variant)
    for p, n in zip(probs, steps):
        b.add(p, cfl=0.8, t_end=1e9, patch_elems=128)
    b.finalize()
    dts = [b.scenario_steps(k)[0] for k in range(len(probs))]
    # explicit step counts: rebuild with the chosen dt
    b.close()
    b = tled.Batch(0)
    b.set_options(graph_steps=40, kernel_variant=variant, batch_schedule=schedule)
    for p, dt, n in zip(probs, dts, steps):
        b.add(p, dt, n, patch_elems=128)
    b.finalize()
    b.run()
    fields = b.read_all()
    for k, (p, dt, n) in enumerate(zip(probs, dts, steps)):
        s = tled.from_problem(p, dt=dt, device=0, kernel_variant=variant, graph_steps=40, patch_elems=128)
        s.step(n)
        assert np.array_equal(fields[k][0], s.read_u()), k
        assert np.array_equal(fields[k][1], s.read_T()), k
        assert fields[k][1].max() > p.params["T0"]
        s.close()
    b.step(30)
    for (u0, T0), (u1, T1) in zip(fields, b.read_all()):
        assert np.array_equal(u0, u1) and np.array_equal(T0, T1)


def test_batch_without_shared_nodes():
    """Scenarios that each fit one patch have no shared node: the shared-node launch is skipped
    (also when timed), and each scenario still equals its own run bit for bit."""
    from paper_2009_10400_amd import tled
    probs = [W.cube_t4(n=2, L=0.01), W.cube_t4(n=3, L=0.012)]
    steps = [30, 55]
    dts = [0.8 * critical_dt(p) for p in probs]
    for gs in (-1, 20):
        b = tled.Batch(0)
        b.set_options(graph_steps=gs)
        for p, dt, n in zip(probs, dts, steps):
            b.add(p, dt, n)
        b.finalize()
        assert b.batch_info()["n_shared_nodes"] == 0
        b.run()
        for k, (p, dt, n) in enumerate(zip(probs, dts, steps)):
            ub, Tb = b.read(k)
            s = tled.from_problem(p, dt=dt, device=0, kernel_variant=2, graph_steps=20, patch_elems=448)
            s.step(n)
            assert np.array_equal(ub, s.read_u()) and np.array_equal(Tb, s.read_T()), (gs, k)
        kt = b.kernel_times(5)
        assert kt["element_ms"] > 0.0 and kt["node_ms"] >= 0.0
        b.close()


def test_batch_through_the_torch_allocator():
    """A batch whose device memory comes from torch's caching allocator gives the same bits."""
    from paper_2009_10400_amd import tled
    sc, steps = small_batch()
    sc, steps = sc[:3], steps[:3]
    out = []
    for ta in (False, True):
        b = tled.Batch(0, use_torch_allocator=ta)
        for (p, _), n in zip(sc, steps):
            b.add(p, 0.8 * critical_dt(p), n)
        b.finalize()
        b.run()
        out.append([f.copy() for pair in b.read_all() for f in pair])
        b.close()
    assert all(np.array_equal(a, c) for a, c in zip(*out))
