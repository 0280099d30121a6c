"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle.

Bar: after 1000 steps, max-abs error of the
displacement relative to max |u| <= 1e-4 and max-abs error of the temperature
<= 0.01 K.  The paper's total error indicators e_u, e_T (Section 6.1) are
printed next to them.
"""
import numpy as np
import pytest

from harness import T_ABS_TOL, U_REL_TOL, errors, gpu_sim, log, one_step_check, oracle_sim, run_parity
from paper_2009_10400_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = [1, 2, 3]


@pytest.mark.parametrize("variant", VARIANTS)
def test_cube_t4_1000_steps(variant):
    """6000-tet cube with a Gaussian source, TI fibre, one Prony term, bottom fixed."""
    err, sim, _ = run_parity(W.cube_t4(), 1000, kernel_variant=variant)
    assert err["u_rel"] <= U_REL_TOL
    assert err["T_abs"] <= T_ABS_TOL
    assert err["u_max"] > 1e-7            # the field is not trivially zero
    assert sim.monitors()["step"] == 1000


@pytest.mark.parametrize("variant", VARIANTS)
def test_cube_h8_1000_steps(variant):
    """12^3 reduced-integration H8 with hourglass control, fibre field, mu(T), 1/r^2 source."""
    p = W.cube_h8(n=12)
    err, sim, _ = run_parity(p, 1000, kernel_variant=variant)
    assert err["u_rel"] <= U_REL_TOL
    assert err["T_abs"] <= T_ABS_TOL


@pytest.mark.parametrize("variant", VARIANTS)
def test_ellipsoid_t4_1000_steps(variant):
    """Jittered, randomly numbered ellipsoid (~30k tets), two Prony terms, line source;
    shrinkage threshold lowered so that it is active."""
    p = W.ellipsoid_t4(30000)
    p.params = dict(p.params, shrink_T=p.params["T0"] + 0.3, shrink_width=1.0)
    err, sim, _ = run_parity(p, 1000, kernel_variant=variant)
    assert err["u_rel"] <= U_REL_TOL
    assert err["T_abs"] <= T_ABS_TOL


PHYSICS = {
    "ti_expansion": dict(expan_mode=1, alpha_m=3e-4),
    "ti_conduction": dict(cond_mode=1, k_m=1.5),
    "ck_of_T": dict(ckT_on=1, ckT_lo=310.15, ckT_hi=312.0),
    "mu_of_T": dict(muT_on=1, muT_lo=310.15, muT_hi=311.0),
    "metabolic_arterial": dict(Q_met=3e4, T_art=311.0),
    "isotropic_no_prony": dict(eta=0.0, g=[], tau=[], n_prony=0),
    "four_prony": dict(g=[0.2, 0.2, 0.1, 0.1], tau=[0.05, 0.2, 1.0, 5.0], n_prony=4),
}


@pytest.mark.parametrize("name", sorted(PHYSICS))
@pytest.mark.parametrize("npe", [4, 8])
def test_physics_variants(name, npe):
    p = W.cube_t4(n=6, L=0.024) if npe == 4 else W.cube_h8(n=8, L=0.04, power=5.0)
    p.params = dict(p.params, **PHYSICS[name])
    err, _, _ = run_parity(p, 400, kernel_variant=2)
    assert err["u_rel"] <= U_REL_TOL
    assert err["T_abs"] <= T_ABS_TOL


def _anisotropic(p, expansion: bool, conduction: bool, seed: int = 17):
    """Orthotropic expansion (Eq. 11: a second axis per element, given with a component along the
    fibre that the library removes) and/or a conductivity tensor per element (Eqs. 15-16: random
    symmetric positive definite, eigenvalues 0.3-1.5 W/(m K))."""
    rng = np.random.default_rng(seed)
    ne = p.ne
    if expansion:
        p.params = dict(p.params, expan_mode=2, alpha_m=3e-4, alpha_n=-1.5e-4)
        a0 = p.a0 if p.a0 is not None else np.tile([1.0, 0.0, 0.0], (ne, 1))
        n = rng.standard_normal((ne, 3))
        p.n0 = n + 0.3 * a0
    if conduction:
        p.params = dict(p.params, cond_mode=2)
        q, r = np.linalg.qr(rng.standard_normal((ne, 3, 3)))
        lam = rng.uniform(0.3, 1.5, (ne, 3))
        p.D = np.einsum("eij,ej,ekj->eik", q, lam, q)
    return p


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("npe", [4, 8])
@pytest.mark.parametrize("mode", ["ortho_expansion", "tensor_conduction", "both_with_kT"])
def test_anisotropic_variants(mode, npe, variant):
    """Orthotropic thermal expansion and per-element conductivity tensors against the oracle,
    all three kernel variants, T4 and H8."""
    p = W.cube_t4(n=6, L=0.024) if npe == 4 else W.cube_h8(n=8, L=0.04, power=5.0)
    p = _anisotropic(p, mode != "tensor_conduction", mode != "ortho_expansion")
    if mode == "both_with_kT":
        p.params = dict(p.params, ckT_on=1, ckT_lo=310.15, ckT_hi=312.0, c_hi=4300.0, k_hi=0.75)
    err, _, _ = run_parity(p, 400, kernel_variant=variant)
    assert err["u_rel"] <= U_REL_TOL
    assert err["T_abs"] <= T_ABS_TOL
    assert err["u_max"] > 1e-8            # the field is not trivially zero


def test_fixed_temperature_and_flipped_elements():
    """Dirichlet T on one face, 30 % of tets given with negative orientation, random numbering."""
    p = W.cube_t4(n=6, L=0.024)
    rng = np.random.default_rng(4)
    flip = rng.random(p.ne) < 0.3
    p.conn[flip] = p.conn[flip][:, [0, 1, 3, 2]]
    onx = np.isclose(p.X[:, 0], 0.0)
    p.fix = p.fix.copy()
    p.fix[onx] |= 8
    p.Tfix = np.full(p.nn, p.params["T0"])
    p.Tfix[onx] = p.params["T0"] + 2.0
    err, sim, _ = run_parity(p, 500, kernel_variant=2)
    assert sim.info()["n_swapped"] == flip.sum()
    assert err["u_rel"] <= U_REL_TOL
    assert err["T_abs"] <= T_ABS_TOL


@pytest.mark.parametrize("npe", [4, 8])
def test_single_element(npe):
    """Smallest mesh: one element, one node fixed (ragged everything)."""
    if npe == 4:
        X = np.array([[0, 0, 0], [0.004, 0, 0], [0.001, 0.0037, 0], [0.0013, 0.0012, 0.0041]])
        conn = np.array([[0, 1, 2, 3]], np.int32)
    else:
        X = W.H8_CORNERS.astype(float) * 0.004
        conn = np.arange(8, dtype=np.int32)[None]
    fix = np.zeros(len(X), np.uint8); fix[0] = 7
    p = W.Problem("single", npe, X, conn, W.base_material(), q=np.array([1e7]), fix=fix)
    for v in VARIANTS:
        err, _, _ = run_parity(p, 300, kernel_variant=v)
        assert err["u_rel"] <= U_REL_TOL and err["T_abs"] <= T_ABS_TOL


def test_monitors_match_oracle():
    p = W.cube_t4()
    sim = gpu_sim(p, kernel_variant=2, graph_steps=25)
    sim.step(200)
    m = sim.monitors()
    o = oracle_sim(p, sim.dt)
    st = o.initial_state(p.params["T0"])
    mon = o.run(st, 200, monitors=True)
    log("  monitors gpu", m, "oracle", mon[-1])
    assert m["step"] == 200
    assert m["strain"] == pytest.approx(mon[-1, 0], rel=1e-3)
    assert m["kinetic"] == pytest.approx(mon[-1, 1], rel=1e-3)
    assert m["T_max"] == pytest.approx(mon[-1, 3], abs=1e-3)
    assert m["T_min"] == pytest.approx(st["T"].min(), abs=1e-3)
    assert m["flags"] == 0


@pytest.mark.parametrize("variant", VARIANTS)
def test_bitwise_determinism_graph_vs_eager(variant):
    p = W.ellipsoid_t4(20000)
    a = gpu_sim(p, kernel_variant=variant, graph_steps=50)
    b = gpu_sim(p, kernel_variant=variant, graph_steps=50)
    c = gpu_sim(p, kernel_variant=variant, graph_steps=-1)
    for s in (a, b, c):
        s.step(230)
    sa, sb, sc = a.read_state(), b.read_state(), c.read_state()
    for k in ("u", "v", "T", "theta"):
        assert np.array_equal(sa[k], sb[k]), k
        assert np.array_equal(sa[k], sc[k]), k


def test_checkpoint_restore_bitwise():
    p = W.cube_h8(n=10)
    s = gpu_sim(p, kernel_variant=2)
    s.step(120)
    blob = s.get_state()
    s.step(150)
    ref = s.read_state()
    s.set_state(blob)
    s.step(150)
    got = s.read_state()
    for k in ("u", "v", "T", "theta"):
        assert np.array_equal(ref[k], got[k]), k
    assert got["step"] == 270


def test_typed_state_roundtrip_and_nan_injection():
    from paper_2009_10400_amd import tled
    p = W.cube_t4(n=5, L=0.02)
    s = gpu_sim(p, kernel_variant=1)
    s.step(50)
    st = s.read_state()
    s.write_state(**{k: st[k] for k in ("u", "v", "T", "theta")}, step=st["step"])
    st2 = s.read_state()
    for k in ("u", "v", "T", "theta"):
        assert np.array_equal(st[k], st2[k]), k
    bad = st["u"].copy()
    free = np.nonzero(p.fix == 0)[0]
    bad[free[0], 0] = np.nan
    s.write_state(u=bad, step=st["step"])
    s.step(3)
    with pytest.raises(tled.TledError) as ei:
        s.sync()
    assert ei.value.status == tled.E_UNSTABLE


def test_errors_surface_through_the_abi():
    from paper_2009_10400_amd import tled
    p = W.cube_t4(n=3, L=0.012)
    s = tled.Sim(0)
    with pytest.raises(tled.TledError) as ei:
        s.step(1)
    assert ei.value.status == tled.E_STATE
    s.set_mesh(4, p.X, p.conn)
    s.set_material(p.params)
    dtc = s.critical_dt()
    s.set_time(3 * dtc, 80.0)
    with pytest.raises(tled.TledError) as ei:
        s.finalize()
    assert ei.value.status == tled.E_ARG
    X = p.X.copy()
    X[p.conn[0]] = X[p.conn[0][0]]          # collapse one element
    s2 = tled.Sim(0)
    s2.set_mesh(4, X, p.conn)
    s2.set_material(p.params)
    s2.set_time(1e-5, 80.0)
    with pytest.raises(tled.TledError) as ei:
        s2.finalize()
    assert ei.value.status == tled.E_MESH


def test_zero_steps_and_all_fixed():
    p = W.cube_t4(n=3, L=0.012)
    p.fix = np.full(p.nn, 7, np.uint8)
    for v in VARIANTS:
        s = gpu_sim(p, kernel_variant=v)
        s.step(0)
        s.sync()
        assert np.all(s.read_u() == 0)
        s.step(100)
        assert np.all(s.read_u() == 0)
        assert s.read_T().max() > p.params["T0"]


def test_device_field_copy_and_torch_allocator():
    import torch
    p = W.cube_t4(n=5, L=0.02)
    s = gpu_sim(p, kernel_variant=2, use_torch_allocator=True)
    s.step(80)
    u_t = torch.zeros((p.nn, 3), dtype=torch.float32, device="cuda:0")
    T_t = torch.zeros(p.nn, dtype=torch.float32, device="cuda:0")
    s.copy_fields_device(u_t, T_t)
    s.sync()
    assert np.array_equal(u_t.cpu().numpy(), s.read_u().astype(np.float32))
    assert np.allclose(T_t.cpu().numpy(), s.read_T(), atol=1e-4)
    info = s.info()
    assert info["device_bytes"] > 0
    assert 1 <= info["patch_wgs_per_cu"] <= 8
    assert info["dt_thermal"] > info["dt"]
    # targets the copy kernel would misread are refused by the binding
    with pytest.raises(ValueError):
        s.copy_fields_device(torch.zeros((p.nn, 3), dtype=torch.float64, device="cuda:0"), None)
    with pytest.raises(ValueError):
        s.copy_fields_device(None, torch.zeros(p.nn - 1, dtype=torch.float32, device="cuda:0"))


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_ellipsoid_one_step(variant):
    """~1.0M-tet ellipsoid in the benchmark's launch configuration: after 60 steps, one more
    step on both sides from the GPU state; increments agree element by element."""
    p = W.ellipsoid_t4(1_000_000)
    p.params = dict(p.params, shrink_T=p.params["T0"] + 0.05, shrink_width=0.5)
    s = gpu_sim(p, kernel_variant=variant)
    r = one_step_check(s, p, n_pre=60)
    log("  full ellipsoid one-step", r)
    assert r["v_rel"] <= 1e-4
    assert r["dT_inc_abs"] <= 1e-5
    assert r["theta_rel"] <= 1e-4


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_h8_one_step(variant):
    """64^3 H8 cube (262k elements) at full size: one-step increments against the oracle."""
    p = W.cube_h8(n=64)
    s = gpu_sim(p, kernel_variant=variant)
    r = one_step_check(s, p, n_pre=60)
    log("  full H8 one-step", r)
    assert r["v_rel"] <= 1e-4
    assert r["dT_inc_abs"] <= 1e-5
    assert r["theta_rel"] <= 1e-4


def test_paper_spheres_liver_material_and_ablation_monitor():
    """Table 5 liver material (T-dependent c and k, metabolic heat, perfusion) with three touching
    uniform spherical sources; the 60 C ablation-zone monitor (lumped volume of nodes at or above
    333.15 K) agrees with the oracle's nodal temperatures."""
    p = W.spheres_t4(n=12, L=0.036)
    sim = gpu_sim(p, kernel_variant=2, ablation_T=310.5, graph_steps=40)
    steps = 800
    sim.step(steps)
    m = sim.monitors()
    u, T = sim.read_u(), sim.read_T()
    o = oracle_sim(p, sim.dt)
    st = o.initial_state(p.params["T0"])
    o.run(st, steps)
    err = errors(st["u"], u, st["T"], T)
    log("  spheres", err, "monitor", m)
    assert err["u_rel"] <= U_REL_TOL and err["T_abs"] <= T_ABS_TOL
    Vl = o.lumped()["Vl"]
    hot = st["T"] >= 310.5
    assert hot.any() and not hot.all()
    margin = np.abs(st["T"] - 310.5) > 1e-3          # nodes sitting on the threshold are ambiguous
    lo, hi = Vl[hot & margin].sum(), Vl[hot | ~margin].sum()
    assert lo - 1e-12 <= m["ablated_volume"] <= hi + 1e-12
