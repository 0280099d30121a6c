"""Shared helpers of the parity tests: run the GPU library and the FP64 oracle
on the same seeded problem and compare with the paper's error measures."""
from __future__ import annotations

import sys
import time

import numpy as np

import oracle
from paper_2009_10400_amd import workloads as W

# Parity bar after 1000 steps: max-abs error of u relative to max |u| <= 1e-4,
# max-abs error of T <= 0.01 K.
U_REL_TOL = 1e-4
T_ABS_TOL = 0.01


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_sim(problem: W.Problem, dt: float) -> oracle.OracleSim:
    return oracle.OracleSim(problem.npe, problem.X, problem.conn, problem.params, a0=problem.a0,
                            q=problem.q, fix=problem.fix, Tfix=problem.Tfix, t_on=problem.t_on,
                            t_off=problem.t_off, dt=dt, gamma=problem.gamma, n0=problem.n0, D=problem.D)


def gpu_sim(problem: W.Problem, dt=None, **opts):
    from paper_2009_10400_amd import tled
    return tled.from_problem(problem, dt=dt, device=0, **opts)


def errors(u_ref, u, T_ref, T):
    """Max-abs errors and the paper's total error indicators e_u, e_T (Section 6.1)."""
    du = np.abs(u - u_ref).max()
    umax = np.abs(u_ref).max()
    dT = np.abs(T - T_ref).max()
    e_u = float(np.sqrt(((u_ref - u) ** 2).sum() / max((u_ref ** 2).sum(), 1e-300)))
    e_T = float(np.sqrt(((T_ref - T) ** 2).sum() / (T_ref ** 2).sum()))
    rng = T_ref.max() - T_ref.min()
    return {"u_rel": float(du / umax) if umax > 0 else float(du), "u_abs": float(du), "u_max": float(umax),
            "T_abs": float(dT), "e_u": e_u, "e_T": e_T,
            "nre_T_max": float(dT / rng) if rng > 0 else 0.0}


def run_parity(problem: W.Problem, steps: int, **opts):
    """Run both sides ``steps`` steps from the initial state; return (errors, gpu sim, oracle state)."""
    t = time.time()
    sim = gpu_sim(problem, **opts)
    dt = sim.dt
    sim.step(steps)
    sim.sync()
    u, T = sim.read_u(), sim.read_T()
    t_gpu = time.time() - t
    t = time.time()
    o = oracle_sim(problem, dt)
    st = o.initial_state(problem.params["T0"])
    if problem.fix is not None and problem.Tfix is not None:
        st["T"][problem.fix & 8 > 0] = problem.Tfix[problem.fix & 8 > 0]
    o.run(st, steps)
    t_orc = time.time() - t
    err = errors(st["u"], u, st["T"], T)
    log(f"  {problem.name} ne={problem.ne} steps={steps} opts={opts} gpu {t_gpu:.2f}s oracle {t_orc:.2f}s -> {err}")
    return err, sim, st


def one_step_check(sim, problem: W.Problem, n_pre: int = 0):
    """Read the GPU state, advance one step on both sides from it, compare the increments."""
    if n_pre:
        sim.step(n_pre)
    s0 = sim.read_state()
    dt = sim.dt
    o = oracle_sim(problem, dt)
    st = {"u": s0["u"].copy(), "u_prev": s0["u"] - dt * s0["v"], "T": s0["T"].copy(),
          "theta": s0["theta"].copy(), "step": s0["step"]}
    o.run(st, 1)
    sim.step(1)
    s1 = sim.read_state()
    dv = np.abs(s1["v"] - (st["u"] - st["u_prev"]) / dt).max()
    vmax = np.abs((st["u"] - st["u_prev"]) / dt).max()
    dTinc = np.abs((s1["T"] - s0["T"]) - (st["T"] - s0["T"])).max()
    Tinc = np.abs(st["T"] - s0["T"]).max()
    th_ref = st["theta"]
    dth = np.abs(s1["theta"] - th_ref).max() if th_ref.size else 0.0
    thmax = np.abs(th_ref).max() if th_ref.size else 1.0
    return {"v_rel": float(dv / vmax) if vmax > 0 else float(dv), "v_max": float(vmax),
            "dT_inc_abs": float(dTinc), "T_inc_max": float(Tinc),
            "theta_rel": float(dth / thmax) if thmax > 0 else float(dth)}
