"""Surrogate-first planning on the GPU, at a size the test suite affords.

A small ensemble is trained on batched solver runs of small planning scenarios;
on held-out scenarios: (1) with the threshold at 0 every scenario falls back and
the result is the solver's, bit for bit; (2) with the calibrated 0.5 K threshold
the accepted scenarios are within the stated bound of the solver and the
surrogate path is faster than the solver alone on the same scenarios.
(The full-size measurement, 2000 training runs and 200 held-out scenarios, is
`bench.py --surrogate 2000`.)"""
import numpy as np
import pytest

from paper_2009_10400_amd import workloads as W

pytestmark = pytest.mark.gpu

DS = 1e-3


@pytest.fixture(scope="module")
def trained():
    from paper_2009_10400_amd import surrogate as S
    train = W.planning_scenarios(80, seed=21, lo=5000, hi=30000, duration_scale=DS)
    calib = W.planning_scenarios(12, seed=22, lo=5000, hi=30000, duration_scale=DS)
    test = W.planning_scenarios(16, seed=23, lo=5000, hi=30000, duration_scale=DS)
    t_ref = 300.0 * DS
    snaps, _ = S.solve_snapshots(train, n_snap=5)
    data = S.make_dataset(train, snaps, t_ref)
    print(f"[planning] {len(snaps)} fields, {len(data.x)} samples", flush=True)
    ens = S.Ensemble(4, t_ref=t_ref)
    hist, secs = ens.fit(data, epochs=30, batch=2048, lr=2e-3)
    print(f"[planning] trained in {secs:.1f}s, final losses {[h[-1] for h in hist]}", flush=True)
    cal, _ = S.solve(calib)
    c = ens.calibrate(calib, cal)
    ref, t_solver = S.solve(test)
    print(f"[planning] calibration factor {c:.3g}; solver alone {t_solver}", flush=True)
    return S, ens, test, ref, t_solver, hist


def test_training_converged(trained):
    S, ens, test, ref, t_solver, hist = trained
    for h in hist:
        assert h[-1] < 0.3 * h[0] and h[-1] < 0.05, h


def test_threshold_zero_falls_back_to_the_solver_bitwise(trained):
    S, ens, test, ref, t_solver, hist = trained
    rep = S.plan(ens, test, threshold_K=0.0)
    assert rep["rejected"] == list(range(len(test)))
    for (kind, u, T), (ur, Tr) in zip(rep["results"], ref):
        assert kind == "solver"
        assert np.array_equal(u, ur) and np.array_equal(T, Tr)


def test_calibrated_plan_accuracy_and_gain(trained):
    S, ens, test, ref, t_solver, hist = trained
    rep = S.plan(ens, test, threshold_K=0.5)
    errs = []
    for k, ((kind, u, T), (ur, Tr)) in enumerate(zip(rep["results"], ref)):
        e = float(np.abs(T - Tr).max())
        errs.append(e)
        if kind == "surrogate":
            # accepted: the calibrated disagreement estimate is within the threshold
            assert rep["estimate"][k] <= 0.5
        else:
            assert np.array_equal(T, Tr)
    acc = [e for (kind, _, _), e in zip(rep["results"], errs) if kind == "surrogate"]
    print(f"[planning] accepted {len(acc)}/{len(test)}, max error accepted "
          f"{max(acc) if acc else None}, all {max(errs):.3f} K; surrogate {rep['t_surrogate']:.3f}s "
          f"+ fallback {rep['t_fallback']['total']:.3f}s vs solver {t_solver['total']:.3f}s", flush=True)
    assert len(acc) >= len(test) // 2
    assert max(acc) <= 0.5               # every accepted scenario within the stated threshold
    assert np.median(errs) <= 0.5
    # the surrogate's GPU work (ensemble inference) is shorter than the solver's GPU work (stepping
    # and read-back) on the same scenarios; at this size both are milliseconds and the end-to-end
    # times are dominated by host set-up, so the end-to-end gain is measured by bench.py
    rep_all = S.plan(ens, test, threshold_K=float("inf"))
    assert not rep_all["rejected"]
    assert rep_all["t_surrogate_gpu"] < t_solver["run"]
