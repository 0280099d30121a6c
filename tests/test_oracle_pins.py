"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it pins.  None of them re-types the oracle's own
tensor formulas: they use hand-derived closed forms, finite differences of the
oracle's separately coded energy, invariants, exact discrete recurrences and
special cases.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2009_10400_amd import workloads as W

MAT = W.base_material()          # mu 1034.48, kappa 1e4, eta 2 mu, alpha 1e-4
T0 = MAT["T0"]


def rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def unit_tet():
    return np.array([[0.0, 0, 0], [0.004, 0, 0], [0.0011, 0.0037, 0], [0.0013, 0.0012, 0.0041]])


def unit_hex(rng=None, jit=0.0):
    X = W.H8_CORNERS.astype(float) * 0.004
    if rng is not None:
        X = X + rng.uniform(-jit, jit, X.shape)
    return X


# ---------------------------------------------------------------- pin 1
def uniaxial_closed_form(s, mu, kappa, eta):
    """Hand-derived S11, S22 of Table 5's model under F = diag(s, 1, 1), fibre along x."""
    S11 = mu * s ** (-2 / 3) * (2 / 3) * (1 - s ** -2) + kappa * (s - 1) / s \
        + (4 / 3) * eta * (s ** (4 / 3) - 1) * s ** (-2 / 3)
    S22 = mu * s ** (-2 / 3) * (1 - s * s) / 3 + kappa * s * (s - 1) \
        - (2 / 3) * eta * (s ** (4 / 3) - 1) * s ** (4 / 3)
    return S11, S22


@pytest.mark.parametrize("s,eta_factor", [(1.1, 2.0), (0.9, 2.0), (1.1, 0.0), (1.3, 2.0), (0.75, 1.0)])
def test_uniaxial_closed_form(s, eta_factor):
    """Table 5 strain energy: uniaxial stretch along the fibre (eta = 0 is Table 1's model)."""
    p = dict(MAT, eta=eta_factor * MAT["mu"])
    S, _ = oracle.stress(p, np.diag([s, 1.0, 1.0]), [1, 0, 0], T0)
    S11, S22 = uniaxial_closed_form(s, p["mu"], p["kappa"], p["eta"])
    assert S[0, 0] == pytest.approx(S11, rel=1e-12, abs=1e-9)
    assert S[1, 1] == pytest.approx(S22, rel=1e-12, abs=1e-9)
    assert S[2, 2] == pytest.approx(S22, rel=1e-12, abs=1e-9)
    off = S - np.diag(np.diag(S))
    assert np.abs(off).max() < 1e-9


def test_uniaxial_closed_form_values():
    """Numbers of the closed form at the cube workload's moduli (mu 1034.4828, kappa 1e4, eta 2 mu)."""
    S, _ = oracle.stress(MAT, np.diag([1.1, 1, 1]), [1, 0, 0], T0)
    assert S[0, 0] == pytest.approx(1372.2166, abs=1e-3)
    assert S[1, 1] == pytest.approx(819.8090, abs=1e-3)
    S, _ = oracle.stress(MAT, np.diag([0.9, 1, 1]), [1, 0, 0], T0)
    assert S[0, 0] == pytest.approx(-1672.5052, abs=1e-3)
    assert S[1, 1] == pytest.approx(-672.6354, abs=1e-3)


@pytest.mark.parametrize("dT", [5.0, 40.0])
def test_uniaxial_with_thermal_pullback(dT):
    """Eq. 10 with isotropic F_th = lambda I: S0 = lambda * S_i(F / lambda)."""
    s = 1.07
    lam = 1 + MAT["alpha"] * dT
    S, _ = oracle.stress(MAT, lam * np.diag([s, 1, 1]), [1, 0, 0], T0 + dT)
    S11, S22 = uniaxial_closed_form(s, MAT["mu"], MAT["kappa"], MAT["eta"])
    assert S[0, 0] == pytest.approx(lam * S11, rel=1e-11)
    assert S[1, 1] == pytest.approx(lam * S22, rel=1e-11)


# ---------------------------------------------------------------- pin 2
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("variant", ["iso_expan", "ti_expan", "muT_shrink"])
def test_stress_is_energy_gradient(seed, variant):
    """First Piola stress F S0 = d(det(Fth) Psi)/dF (Eqs. 9-10), central differences."""
    rng = np.random.default_rng(seed)
    p = dict(MAT)
    if variant == "ti_expan":
        p.update(expan_mode=1, alpha_m=4e-4)
    if variant == "muT_shrink":
        p.update(muT_on=1, shrink_on=1)
    F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
    if np.linalg.det(F) < 0.2:
        F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
    a0 = rng.standard_normal(3)
    Te = T0 + rng.uniform(0, 30)
    S, _ = oracle.stress(p, F, a0, Te)
    P = F @ S
    h = 1e-6
    G = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            Fp = F.copy(); Fp[i, j] += h
            Fm = F.copy(); Fm[i, j] -= h
            G[i, j] = (oracle.stress(p, Fp, a0, Te)[1] - oracle.stress(p, Fm, a0, Te)[1]) / (2 * h)
    assert np.abs(P - G).max() <= 1e-6 * max(1.0, np.abs(P).max())
    assert np.abs(S - S.T).max() <= 1e-9 * max(1.0, np.abs(S).max())


# ---------------------------------------------------------------- pin 3
@pytest.mark.parametrize("npe", [4, 8])
@pytest.mark.parametrize("seed", range(3))
def test_nodal_force_is_energy_gradient(npe, seed):
    """f_a = d/du_a [V0 det(Fth) Psi + hourglass energy] at fixed T (Eqs. 24-26, 10)."""
    rng = np.random.default_rng(100 + seed)
    p = dict(MAT, n_prony=0, g=[], tau=[])
    Xe = unit_tet() if npe == 4 else unit_hex(rng, 3e-4)
    ue = 2e-4 * rng.standard_normal((npe, 3))
    Te = T0 + rng.uniform(0, 20, npe)
    a0 = rng.standard_normal(3)
    f, _, _ = oracle.element(p, Xe, ue, Te, a0)
    h = 1e-9
    G = np.zeros_like(ue)
    for a in range(npe):
        for i in range(3):
            up = ue.copy(); up[a, i] += h
            um = ue.copy(); um[a, i] -= h
            G[a, i] = (oracle.element(p, Xe, up, Te, a0)[2] - oracle.element(p, Xe, um, Te, a0)[2]) / (2 * h)
    assert np.abs(f - G).max() <= 2e-5 * np.abs(f).max()


# ---------------------------------------------------------------- pins 4, 5, 6
@pytest.mark.parametrize("npe", [4, 8])
def test_rigid_rotation_free_expansion(npe):
    """u = (lambda R - I) X with uniform T: zero stress and zero nodal force (Eqs. 7-10)."""
    rng = np.random.default_rng(7)
    Xe = unit_tet() if npe == 4 else unit_hex(rng, 3e-4)
    for dT, ang in [(0.0, 0.7), (25.0, 0.0), (25.0, 1.9)]:
        lam = 1 + MAT["alpha"] * dT
        R = rot([1, 2, 3], ang)
        ue = Xe @ (lam * R - np.eye(3)).T
        p = dict(MAT, hg_coef=0.0) if npe == 8 else MAT
        f, h, e = oracle.element(p, Xe, ue, T0 + dT, [0.3, 0.5, 0.8])
        assert np.abs(f).max() < 1e-12
        assert abs(e) < 1e-15


def test_clamped_uniform_heating():
    """F = I, uniform heating: S0 = kappa (lambda^-3 - 1) I; -29.940 Pa at 10 K, -148.512 Pa at 50 K."""
    for dT, ref in [(10.0, -29.940), (50.0, -148.512)]:
        S, _ = oracle.stress(MAT, np.eye(3), [1, 0, 0], T0 + dT)
        lam = 1 + MAT["alpha"] * dT
        assert np.allclose(S, MAT["kappa"] * (lam ** -3 - 1) * np.eye(3), rtol=1e-12, atol=1e-12)
        assert S[0, 0] == pytest.approx(ref, abs=1e-3)
    # element: f_a = V0 S0 dh_a/dX, so the forces balance
    f, h, _ = oracle.element(MAT, unit_tet(), np.zeros((4, 3)), T0 + 10, [1, 0, 0])
    assert np.abs(f.sum(0)).max() < 1e-12 * np.abs(f).max()


# ---------------------------------------------------------------- pin 7
def _box(kind, n, L):
    X, conn, h = W.box_mesh(kind, n, L)
    return X, conn


@pytest.mark.parametrize("kind,npe", [("t4", 4), ("h8", 8)])
@pytest.mark.parametrize("stretch", [1.0, 1.3])
@pytest.mark.parametrize("ang", [0.0, 0.8])
def test_linear_conduction_patch(kind, npe, stretch, ang):
    """Linear T, no sources: zero load off the two x faces; face totals +-k A0 dT / (s L0)
    (Eqs. 15-19: pulled-back conduction K0 = J k C^-1; rotation does not change it)."""
    L, n = 0.02, 4
    X, conn = _box(kind, n, L)
    p = dict(MAT, alpha=0.0, alpha_m=0.0)
    s = oracle.OracleSim(npe, X, conn, p, dt=1e-3)
    G = 500.0  # K/m
    T = T0 + G * X[:, 0]
    Fdef = rot([0.2, 1, 0.4], ang) @ np.diag([stretch, 1, 1])
    u = X @ (Fdef - np.eye(3)).T
    _, H = s.loads(u, T)
    on0 = np.isclose(X[:, 0], 0.0)
    onL = np.isclose(X[:, 0], L)
    inner = ~(on0 | onL)
    flux = MAT["k"] * L * L * G / stretch
    assert np.abs(H[inner]).max() < 1e-12 * flux
    assert H[onL].sum() == pytest.approx(flux, rel=1e-10)
    assert H[on0].sum() == pytest.approx(-flux, rel=1e-10)


def test_transient_conduction_converges_to_linear_profile():
    """Dirichlet T at x = 0 and x = L, adiabatic elsewhere: explicit Pennes (Eq. 20, minus sign
    on conduction) converges to the linear steady profile."""
    L, n = 0.01, 4
    X, conn = _box("t4", n, L)
    p = dict(MAT, alpha=0.0, alpha_m=0.0, wbcb=0.0, g=[], tau=[], n_prony=0)
    fix = np.zeros(len(X), np.uint8)
    Tfix = np.zeros(len(X))
    on0 = np.isclose(X[:, 0], 0.0)
    onL = np.isclose(X[:, 0], L)
    fix[on0 | onL] = 8
    Tfix[on0] = T0
    Tfix[onL] = T0 + 10.0
    dt = 2.0
    s = oracle.OracleSim(4, X, conn, p, fix=fix, Tfix=Tfix, dt=dt)
    st = s.initial_state(T0)
    s.run(st, 1500)
    exact = T0 + 10.0 * X[:, 0] / L
    assert np.abs(st["T"] - exact).max() < 1e-6
    assert np.all(st["u"] == 0.0)


# ---------------------------------------------------------------- pin 8
def test_pennes_0d_closed_form():
    """Uniform T and source: T^n - T_eq = (1 - dt w_b c_b / (rho c))^n (T^0 - T_eq), Eq. 20."""
    X, conn = _box("t4", 3, 0.01)
    Q = 2e5
    p = dict(MAT, alpha=0.0, alpha_m=0.0)
    dt = 0.05
    s = oracle.OracleSim(4, X, conn, p, q=np.full(len(conn), Q), dt=dt)
    st = s.initial_state(T0)
    n = 400
    s.run(st, n)
    w = p["wbcb"]
    Teq = p["T_art"] + Q / w
    ref = Teq + (1 - dt * w / (p["rho"] * p["c"])) ** n * (T0 - Teq)
    assert np.abs(st["T"] - ref).max() < 1e-9


def test_pennes_no_perfusion_rise():
    """No perfusion: per-step rise exactly Q dt / (rho c) (the 0.04 m cube: 5e7 W/m^3 -> 7.089e-3 K/step at 5.104e-4 s)."""
    X, conn = _box("h8", 2, 0.01)
    p = dict(MAT, alpha=0.0, alpha_m=0.0, wbcb=0.0)
    dt = 5.104e-4
    s = oracle.OracleSim(8, X, conn, p, q=np.full(len(conn), 5e7), dt=dt)
    st = s.initial_state(T0)
    s.run(st, 10)
    assert np.allclose(st["T"] - T0, 10 * 5e7 * dt / (p["rho"] * p["c"]), rtol=1e-12)
    assert 5e7 * dt / 3.6e6 == pytest.approx(7.089e-3, abs=1e-6)


# ---------------------------------------------------------------- pin 9
@pytest.mark.parametrize("g,tau", [([0.5], [0.5]), ([0.3, 0.2], [0.1, 2.0])])
def test_prony_step_relaxation(g, tau):
    """Held strain: S~^n / S0 = 1 - sum g_i (1 - b_i^n), b_i = tau_i / (dt + tau_i) (recursion after Eq. 27)."""
    p = dict(MAT, g=g, tau=tau, n_prony=len(g))
    dt = 5.1038e-4
    Xe = unit_tet()
    ue = np.array([[0, 0, 0], [1e-4, 0, 0], [2e-5, 3e-5, 0], [0, 1e-5, -4e-5]])
    f_el, _, _ = oracle.element(dict(p, n_prony=0, g=[], tau=[]), Xe, ue, T0, [1, 0, 0])
    theta = np.zeros(6 * len(g))
    for n in range(1, 1001):
        f, _, _ = oracle.element(p, Xe, ue, T0, [1, 0, 0], theta=theta, dt=dt)
        if n in (1, 10, 1000):
            ratio = 1 - sum(gi * (1 - (ti / (dt + ti)) ** n) for gi, ti in zip(g, tau))
            assert np.allclose(f, ratio * f_el, rtol=1e-10, atol=1e-14 * np.abs(f_el).max())
    if len(g) == 1:
        cd = math.sqrt((MAT["kappa"] + 4 * MAT["mu"] / 3 + 4 * MAT["eta"]) / MAT["rho"])
        dt_cube = 0.8 * (0.004 / math.sqrt(2)) / cd       # the 0.04 m cube's step, 5.1038e-4 s
        b = 0.5 / (dt_cube + 0.5)
        assert b ** 1000 == pytest.approx(0.360506, abs=2e-6)
        assert 1 - 0.5 * (1 - b ** 1000) == pytest.approx(0.680253, abs=2e-6)
        # dt -> 0 limit is the generalised Maxwell relaxation exp(-t / tau)
        assert (0.5 / (1e-7 + 0.5)) ** round(0.51038 / 1e-7) == pytest.approx(math.exp(-0.51038 / 0.5), rel=1e-6)


# ---------------------------------------------------------------- pin 10
@pytest.mark.parametrize("npe", [4, 8])
def test_element_balance_invariants(npe):
    """Per element: sum_a f_a = 0, sum_a h_a = 0, sum_a x_a x f_a = 0 (T4; H8 without hourglass)."""
    rng = np.random.default_rng(3)
    for trial in range(5):
        Xe = unit_tet() if npe == 4 else unit_hex(rng, 4e-4)
        ue = 5e-4 * rng.standard_normal((npe, 3))
        Te = T0 + rng.uniform(0, 30, npe)
        p = dict(MAT, hg_coef=0.0)
        f, h, _ = oracle.element(p, Xe, ue, Te, rng.standard_normal(3))
        sc = np.abs(f).max()
        assert np.abs(f.sum(0)).max() < 1e-12 * sc
        assert abs(h.sum()) < 1e-12 * np.abs(h).max()
        x = Xe + ue
        assert np.abs(np.cross(x, f).sum(0)).max() < 1e-12 * sc * 0.01


def test_hourglass_vanishes_on_affine_fields():
    """Hourglass control only resists the zero-energy modes: none on u = A X + b, some on h-modes."""
    rng = np.random.default_rng(4)
    Xe = unit_hex(rng, 5e-4)
    A = 1e-2 * rng.standard_normal((3, 3))
    ue = Xe @ A.T + 1e-3
    f1, _, e1 = oracle.element(dict(MAT, hg_coef=0.1), Xe, ue, T0, [1, 0, 0])
    f0, _, e0 = oracle.element(dict(MAT, hg_coef=0.0), Xe, ue, T0, [1, 0, 0])
    assert np.abs(f1 - f0).max() < 1e-12 * np.abs(f0).max()
    assert e1 == pytest.approx(e0, rel=1e-12)
    # an hourglass mode: xi*eta pattern in u_z gives no strain at the centre but hourglass energy
    hmode = (W.H8_CORNERS[:, 0] * 2 - 1) * (W.H8_CORNERS[:, 1] * 2 - 1)
    ue = np.zeros((8, 3)); ue[:, 2] = 1e-5 * hmode
    Xr = W.H8_CORNERS.astype(float) * 0.004
    f0, _, e0 = oracle.element(dict(MAT, hg_coef=0.0), Xr, ue, T0, [1, 0, 0])
    f1, _, e1 = oracle.element(dict(MAT, hg_coef=0.1), Xr, ue, T0, [1, 0, 0])
    assert np.abs(f0).max() < 1e-15 and e1 > 0
    assert np.abs(f1.sum(0)).max() < 1e-12 * np.abs(f1).max()


@pytest.mark.parametrize("L", [0.004, 0.01])
def test_hourglass_closed_form_on_a_cube(L):
    """The hourglass term as read for H8 elements (the paper only cites its source): on an
    undistorted cube of side L the hourglass vectors reduce to the base vectors h (X^T h = 0),
    every |dh_a/dX|^2 is 3/(16 L^2) at the centre, so k = 3 c (kappa + 4 mu / 3) L / 16, and the
    mode u = a h e_i (which the one-point strain does not see) stores 32 k a^2 = 6 c (kappa +
    4 mu / 3) L a^2 with nodal forces 8 k a h e_i.  Modes are orthogonal: energies add."""
    c = 0.1
    Xr = W.H8_CORNERS.astype(float) * L
    xi, eta, zeta = (2 * W.H8_CORNERS.T - 1).astype(float)
    modes = [xi * eta, eta * zeta, zeta * xi, xi * eta * zeta]
    kk = 3 * c * (MAT["kappa"] + 4 * MAT["mu"] / 3) * L / 16
    a = 1e-6
    total_u, total_e = np.zeros((8, 3)), 0.0
    for m, h in enumerate(modes):
        for i in range(3):
            ue = np.zeros((8, 3)); ue[:, i] = a * h
            f, _, e = oracle.element(dict(MAT, hg_coef=c), Xr, ue, T0, [1, 0, 0])
            assert e == pytest.approx(32 * kk * a * a, rel=1e-9)
            fref = np.zeros((8, 3)); fref[:, i] = 8 * kk * a * h
            assert np.abs(f - fref).max() <= 1e-9 * np.abs(fref).max()
        # one mode per direction, summed: the energies add
        total_u[:, m % 3] += (m + 1) * a * h
        total_e += 32 * kk * ((m + 1) * a) ** 2
    _, _, e = oracle.element(dict(MAT, hg_coef=c), Xr, total_u, T0, [1, 0, 0])
    assert e == pytest.approx(total_e, rel=1e-9)


def test_global_momentum_and_heat_conservation():
    """No fixed dofs, no perfusion: sum M v stays 0 and sum C T is conserved (sum_e of Eqs. 14, 23)."""
    X, conn, h = W.box_mesh("t4", 4, 0.02)
    p = dict(MAT, wbcb=0.0)
    rng = np.random.default_rng(0)
    s = oracle.OracleSim(4, X, conn, p, dt=2e-4, gamma=0.0)
    st = s.initial_state(T0)
    st["T"] = T0 + 20 * rng.random(len(X))
    mon = s.run(st, 200, monitors=True)
    M = s.lumped()["M"]
    mom = (M[:, None] * (st["u"] - st["u_prev"])).sum(0)
    assert np.abs(mom).max() < 1e-14 * (M[:, None] * np.abs(st["u"] - st["u_prev"])).sum()
    heat0 = (p["rho"] * p["c"] * s.lumped()["Vl"] * (T0 + 0 * X[:, 0])).sum()
    assert mon[-1, 4] == pytest.approx(mon[0, 4], rel=1e-14)
    assert np.abs(st["u"]).max() > 0


# ---------------------------------------------------------------- pin 11
@pytest.mark.parametrize("kind,npe", [("t4", 4), ("h8", 8)])
def test_energy_conservation_undamped(kind, npe):
    """gamma = 0, no Prony, isothermal, free body: E = 1/2 v^- M v^+ + strain energy is conserved
    to 1e-3 over 1000 steps at 0.8 of the critical step (central difference, Eq. 27)."""
    X, conn, h = W.box_mesh(kind, 4, 0.02)
    rng = np.random.default_rng(11)
    X = X + np.where((X > 0) & (X < 0.02), 0.15 * h, 0) * rng.uniform(-1, 1, X.shape)
    p = dict(MAT, n_prony=0, g=[], tau=[], wbcb=0.0)
    s0 = oracle.OracleSim(npe, X, conn, p, dt=1e-4)
    dt = 0.8 * s0.critical_dt
    s = oracle.OracleSim(npe, X, conn, p, dt=dt, gamma=0.0)
    st = s.initial_state(T0)
    st["u"] = 1e-4 * h * rng.standard_normal(X.shape)
    st["u_prev"] = st["u"].copy()
    mon = s.run(st, 1000, monitors=True)
    E = mon[:, 0] + mon[:, 2]
    assert np.abs(E - E[0]).max() / E[0] <= 1e-3
    assert mon[:, 1].max() > 0.1 * E[0]      # energy actually oscillates between the two forms


def test_rigid_translation_damping():
    """Force-free rigid motion with mass-proportional damping D = gamma M (Eqs. 21-22):
    v decays like exp(-gamma t) up to the scheme's O((gamma dt)^3) per-step error."""
    X, conn, h = W.box_mesh("t4", 2, 0.01)
    gamma, dt = 80.0, 5e-4
    s = oracle.OracleSim(4, X, conn, dict(MAT, alpha=0.0), dt=dt, gamma=gamma)
    st = s.initial_state(T0)
    v0 = np.array([1e-3, -2e-3, 5e-4])
    st["u"] = np.tile(v0 * dt, (len(X), 1))
    n = 100
    s.run(st, n)
    v = (st["u"] - st["u_prev"]) / dt
    exact = v0 * math.exp(-gamma * n * dt)
    assert np.abs(v - exact).max() < n * (gamma * dt) ** 3 / 12 * np.abs(v0).max() * 1.5


# ---------------------------------------------------------------- pin 12
def test_no_expansion_gives_zero_displacement():
    """alpha = 0 (the paper's temperature-independent, no-expansion case, Table 6 row 1): u == 0 bitwise."""
    p = W.cube_t4(n=4, L=0.016)
    prm = dict(p.params, alpha=0.0, alpha_m=0.0)
    s = oracle.OracleSim(4, p.X, p.conn, prm, a0=p.a0, q=p.q, fix=p.fix, dt=4e-4, gamma=80)
    st = s.initial_state(T0)
    s.run(st, 50)
    assert np.all(st["u"] == 0.0)
    assert st["T"].max() > T0 + 0.1


def test_orientation_repair_and_permutation_invariance():
    """Flipped T4 (negative volume) are repaired by swapping the last two nodes; node/element order
    does not change the physics."""
    p = W.cube_t4(n=3, L=0.012)
    rng = np.random.default_rng(2)
    conn = p.conn.copy()
    flip = rng.random(len(conn)) < 0.3
    conn[flip] = conn[flip][:, [0, 1, 3, 2]]
    pe = rng.permutation(len(conn))
    pn = rng.permutation(p.nn)
    inv = np.empty_like(pn); inv[pn] = np.arange(p.nn)
    kw = dict(dt=4e-4, gamma=80)
    s1 = oracle.OracleSim(4, p.X, p.conn, p.params, a0=p.a0, q=p.q, fix=p.fix, **kw)
    s2 = oracle.OracleSim(4, p.X[pn], inv[conn[pe]], p.params, a0=p.a0[pe], q=p.q[pe], fix=p.fix[pn], **kw)
    assert s2.n_swapped == flip.sum() and s1.n_swapped == 0
    a, b = s1.initial_state(T0), s2.initial_state(T0)
    s1.run(a, 30); s2.run(b, 30)
    assert np.abs(a["u"][pn] - b["u"]).max() < 1e-9 * np.abs(a["u"]).max()   # summation order only
    assert np.allclose(a["T"][pn], b["T"], rtol=0, atol=1e-10)


# ---------------------------------------------------------------- pin 14
@pytest.mark.parametrize("kind,npe", [("t4", 4), ("h8", 8)])
def test_mass_invariants(kind, npe):
    """Lumped matrices conserve mass (Section 4.2): sum M = rho V, sum C = rho c V, sum Qr = sum q V0."""
    X, conn, h = W.box_mesh(kind, 5, 0.04)
    q = np.linspace(1, 2, len(conn)) * 1e5
    s = oracle.OracleSim(npe, X, conn, MAT, q=q, dt=1e-4)
    L = s.lumped()
    _, _, V0 = s.geometry()
    assert V0.sum() == pytest.approx(0.04 ** 3, rel=1e-12)
    assert L["M"].sum() == pytest.approx(MAT["rho"] * 0.04 ** 3, rel=1e-12)
    assert L["Kb"].sum() == pytest.approx(MAT["wbcb"] * 0.04 ** 3, rel=1e-12)
    assert L["Qr"].sum() == pytest.approx((q * V0).sum(), rel=1e-12)
    assert np.all(V0 > 0)


def _stability_limits(npe, jitter):
    """Exact limits of a small box (2^3 cells, 8 mm): the undamped central-difference step 2/omega_max
    with omega^2 the eigenvalues of M^-1 K, K the internal-force Jacobian at u = 0 by central
    differences of the oracle's loads (elastic, fibre and hourglass stiffness included), and the
    explicit heat step 2/lambda_max of C^-1 K_T likewise."""
    X, conn, h = W.box_mesh("t4" if npe == 4 else "h8", 2, 0.008)
    if jitter:
        inner = np.all((X > 1e-9) & (X < 0.008 - 1e-9), axis=1)
        X = X + jitter * h * np.random.default_rng(1).uniform(-1, 1, X.shape) * inner[:, None]
    s = oracle.OracleSim(npe, X, conn, dict(MAT, hg_coef=0.1), dt=1e-5)
    nn = X.shape[0]
    T = np.full(nn, T0)
    K = np.zeros((3 * nn, 3 * nn))
    for j in range(3 * nn):
        u = np.zeros((nn, 3)); u.flat[j] = 1e-9
        Fp, _ = s.loads(u, T)
        u.flat[j] = -1e-9
        Fm, _ = s.loads(u, T)
        K[:, j] = (Fp - Fm).ravel() / 2e-9
    m = np.repeat(1 / np.sqrt(s.lumped()["M"]), 3)
    A = m[:, None] * K * m[None, :]
    w2 = np.linalg.eigvalsh(0.5 * (A + A.T)).max()
    KT = np.zeros((nn, nn))
    for j in range(nn):
        Tp, Tm = T.copy(), T.copy()
        Tp[j] += 1e-6; Tm[j] -= 1e-6
        KT[:, j] = (s.loads(np.zeros((nn, 3)), Tp)[1] - s.loads(np.zeros((nn, 3)), Tm)[1]) / 2e-6
    c = 1 / np.sqrt(MAT["rho"] * MAT["c"] * s.lumped()["Vl"])
    B = c[:, None] * KT * c[None, :]
    lt = np.linalg.eigvalsh(0.5 * (B + B.T)).max()
    return s.critical_dt, 2 / np.sqrt(w2), 2 / lt


@pytest.mark.parametrize("npe", [4, 8])
@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_critical_step_is_stable(npe, jitter):
    """The critical step as read (min_e L_e / c_d, c_d with the fibre stiffness) against the exact
    stability limits of the discrete system (Eq. 27 and the explicit heat update of Eq. 20): below
    the undamped mechanical limit, within a factor of two of it, and far below the thermal one."""
    dt_cr, dt_mech, dt_heat = _stability_limits(npe, jitter)
    assert 0.5 * dt_mech <= dt_cr <= dt_mech
    assert dt_cr < 1e-3 * dt_heat


def test_c1_critical_step():
    """6000-tet cube (h = 4 mm): 0.8 * min L_e / c_d = 5.104e-4 s (Kuhn tet L = 3 V / A_max = h / sqrt 2)."""
    p = W.cube_t4()
    s = oracle.OracleSim(4, p.X, p.conn, p.params, dt=1e-4)
    cd = math.sqrt((MAT["kappa"] + 4 * MAT["mu"] / 3 + 4 * MAT["eta"]) / MAT["rho"])
    assert s.critical_dt == pytest.approx((0.004 / math.sqrt(2)) / cd, rel=1e-12)
    assert 0.8 * s.critical_dt == pytest.approx(5.104e-4, abs=1e-7)
