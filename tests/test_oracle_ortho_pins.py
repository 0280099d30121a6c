"""Pins of the oracle's orthotropic thermal expansion (Eq. 11) and of a general
element conductivity tensor in the pulled-back conduction (Eqs. 15-16).

Expected values come from derivations written here: the exact stress-free
state u = (F_th - I) X, the purely volumetric response of a clamped body (which
is hydrostatic whatever the axes), the diagonal-stretch closed form of Table 5's
model, frame indifference when the material axes rotate together, and the first
moment of consistent nodal loads of a uniform flux.  Readings: the first
expansion axis m is the fibre a0; the second axis n is made orthonormal to m
(Gram-Schmidt); the element tensor D is the conductivity of Eq. 15 as given
(constant in time; scaled by k(T)/k when c(T), k(T) are on).
``tests/test_oracle_mutations.py`` plants mistakes in these laws and checks
that these tests catch them.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2009_10400_amd import workloads as W

MAT = W.base_material()          # mu 1034.48, kappa 1e4, eta 2 mu, alpha 1e-4
T0 = MAT["T0"]
ORTHO = dict(MAT, expan_mode=2, alpha=1e-4, alpha_m=4e-4, alpha_n=-2e-4)


def unit_tet():
    return np.array([[0.0, 0, 0], [0.004, 0, 0], [0.0011, 0.0037, 0], [0.0013, 0.0012, 0.0041]])


def unit_hex(rng, jit=3e-4):
    return W.H8_CORNERS.astype(float) * 0.004 + rng.uniform(-jit, jit, (8, 3))


def rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def stretches(p, dT):
    return 1 + p["alpha"] * dT, 1 + p["alpha_m"] * dT, 1 + p["alpha_n"] * dT


# ---------------------------------------------------------------- orthotropic expansion, Eq. 11
@pytest.mark.parametrize("npe", [4, 8])
@pytest.mark.parametrize("seed", range(3))
def test_ortho_expansion_free(npe, seed):
    """u = (F_th - I) X with F_th = l_i I + (l_m - l_i) m m + (l_n - l_i) n n (three different
    ratios) is the stress-free intermediate state (Eqs. 7-8): zero nodal force.  The second axis
    is passed with a component along m, which the oracle removes (orthonormal axes)."""
    rng = np.random.default_rng(70 + seed)
    Xe = unit_tet() if npe == 4 else unit_hex(rng)
    R = rotation(rng)
    m, n = R[:, 0], R[:, 1]
    dT = rng.uniform(5, 40)
    li, lm, ln = stretches(ORTHO, dT)
    Fth = li * np.eye(3) + (lm - li) * np.outer(m, m) + (ln - li) * np.outer(n, n)
    ue = Xe @ (Fth - np.eye(3)).T
    n_raw = 2.5 * n + 0.7 * m
    f, _, e = oracle.element(ORTHO, Xe, ue, T0 + dT, m, n0=n_raw)
    scale = ORTHO["kappa"] * 4e-4 * 0.004 ** 2
    assert np.abs(f).max() < 1e-11 * scale
    assert abs(e) < 1e-18
    # the same displacement with the m and n ratios exchanged is not stress-free
    Fsw = li * np.eye(3) + (ln - li) * np.outer(m, m) + (lm - li) * np.outer(n, n)
    f2, _, _ = oracle.element(ORTHO, Xe, Xe @ (Fsw - np.eye(3)).T, T0 + dT, m, n0=n_raw)
    assert np.abs(f2).max() > 1e-3 * scale


@pytest.mark.parametrize("seed", range(3))
def test_ortho_clamped_volumetric(seed):
    """Clamped (F = I), mu = eta = 0: F_e = F_th^-1, C_e^-1 = F_th^2 and
    S0 = det F_th F_th^-1 kappa J (J - 1) F_th^2 F_th^-T = kappa ((l_i l_m l_n)^-1 - 1) I,
    hydrostatic for any orientation of the axes (Eqs. 9-11)."""
    rng = np.random.default_rng(80 + seed)
    R = rotation(rng)
    p = dict(ORTHO, mu=0.0, eta=0.0)
    dT = 25.0
    li, lm, ln = stretches(p, dT)
    S, _ = oracle.stress(p, np.eye(3), R[:, 0], T0 + dT, n0=R[:, 1])
    assert np.allclose(S, p["kappa"] * (1 / (li * lm * ln) - 1) * np.eye(3), rtol=1e-12, atol=1e-9)


def diag_stress(p_, q_, r_, mu, kappa, eta):
    """S_i of Table 5's model for F_e = diag(p, q, r), fibre along x, by hand:
    C = diag(p^2, q^2, r^2), J = p q r, I1 = p^2 + q^2 + r^2, I4 = p^2, c = J^(-2/3);
    S_kk = mu c (1 - I1 / (3 C_kk)) + 2 eta (c I4 - 1) c (delta_k1 - I4 / (3 C_kk)) + kappa J (J - 1) / C_kk."""
    Ck = np.array([p_ * p_, q_ * q_, r_ * r_])
    J = p_ * q_ * r_
    c = J ** (-2.0 / 3.0)
    I1, I4 = Ck.sum(), Ck[0]
    e1 = np.array([1.0, 0.0, 0.0])
    return mu * c * (1 - I1 / (3 * Ck)) + 2 * eta * (c * I4 - 1) * c * (e1 - I4 / (3 * Ck)) + kappa * J * (J - 1) / Ck


def test_diag_stress_helper_matches_uniaxial():
    """Self-check of the helper against the uniaxial closed form (pin 1, 1.1 stretch: S11 1372.2166,
    S22 819.8090 Pa)."""
    S = diag_stress(1.1, 1.0, 1.0, MAT["mu"], MAT["kappa"], MAT["eta"])
    assert S[0] == pytest.approx(1372.2166, abs=1e-3)
    assert S[1] == pytest.approx(819.8090, abs=1e-3) and S[2] == pytest.approx(S[1], rel=1e-14)


@pytest.mark.parametrize("dT", [10.0, 30.0])
def test_ortho_clamped_heating_axes(dT):
    """F = I, m = e_x (also the fibre), n = e_y: F_th = diag(l_m, l_n, l_i), F_e = diag(1/l_m, 1/l_n, 1/l_i),
    and the pull-back of Eq. 10 gives S0_kk = l_i l_m l_n S_i,kk / F_th,kk^2."""
    li, lm, ln = stretches(ORTHO, dT)
    S, _ = oracle.stress(ORTHO, np.eye(3), [1, 0, 0], T0 + dT, n0=[0, 1, 0])
    Si = diag_stress(1 / lm, 1 / ln, 1 / li, ORTHO["mu"], ORTHO["kappa"], ORTHO["eta"])
    ref = li * lm * ln * Si / np.array([lm, ln, li]) ** 2
    assert np.allclose(np.diag(S), ref, rtol=1e-10)
    assert np.abs(S - np.diag(np.diag(S))).max() < 1e-10


def test_ortho_clamped_heating_values():
    """The numbers at dT = 30 K (alpha 1e-4, 4e-4, -2e-4 across, along m, along n):
    S0 = diag(-155.8677, -45.5705, -64.5557) Pa (from the diagonal closed form above)."""
    S, _ = oracle.stress(ORTHO, np.eye(3), [1, 0, 0], T0 + 30.0, n0=[0, 1, 0])
    assert np.diag(S) == pytest.approx([-155.8677, -45.5705, -64.5557], abs=2e-4)


@pytest.mark.parametrize("seed", range(3))
def test_ortho_frame_indifference(seed):
    """Rotating the deformation and both material axes together rotates the stress:
    S0(R F R^T; R m, R n) = R S0(F; m, n) R^T (Table 5's model with Eq. 11 is built from
    invariants of C_e and the axes)."""
    rng = np.random.default_rng(90 + seed)
    R = rotation(rng)
    F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
    m = np.array([1.0, 0.0, 0.0])
    n = np.array([0.0, 1.0, 0.0])
    S, psi = oracle.stress(ORTHO, F, m, T0 + 20.0, n0=n)
    Sr, psir = oracle.stress(ORTHO, R @ F @ R.T, R @ m, T0 + 20.0, n0=R @ n)
    assert np.allclose(Sr, R @ S @ R.T, rtol=1e-10, atol=1e-9)
    assert psir == pytest.approx(psi, rel=1e-10)


def test_ortho_reduces_to_transversely_isotropic():
    """alpha_n = alpha gives l_n = l_i: Eq. 11 reduces to its transversely isotropic form."""
    rng = np.random.default_rng(7)
    F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
    R = rotation(rng)
    S2, _ = oracle.stress(dict(ORTHO, alpha_n=ORTHO["alpha"]), F, R[:, 0], T0 + 25.0, n0=R[:, 1])
    S1, _ = oracle.stress(dict(ORTHO, expan_mode=1), F, R[:, 0], T0 + 25.0)
    assert np.allclose(S2, S1, rtol=1e-12, atol=1e-10)


def test_ortho_parallel_axes_rejected():
    """n parallel to m defines no orthotropic frame: set-up refuses it."""
    X, conn, _ = W.box_mesh("t4", 1, 0.01)
    a0 = np.tile([1.0, 0.0, 0.0], (len(conn), 1))
    with pytest.raises(ValueError):
        oracle.OracleSim(4, X, conn, ORTHO, a0=a0, n0=2.0 * a0, dt=1e-3)
    with pytest.raises(ValueError):
        oracle.OracleSim(4, X, conn, ORTHO, a0=a0, dt=1e-3)        # n0 missing


# ---------------------------------------------------------------- conductivity tensor, Eqs. 15-16
TEN = dict(MAT, alpha=0.0, alpha_m=0.0, cond_mode=2, k=0.5)


def spd(rng, k=(0.4, 0.9, 1.6)):
    R = rotation(rng)
    return R @ np.diag(k) @ R.T


def first_moment(kind, npe, D, u_of_X, G):
    L, n = 0.02, 4
    X, conn, _ = W.box_mesh(kind, n, L)
    s = oracle.OracleSim(npe, X, conn, TEN, D=np.tile(D, (len(conn), 1, 1)), dt=1e-3)
    _, H = s.loads(u_of_X(X), T0 + X @ G)
    interior = np.all((X > 1e-9) & (X < L - 1e-9), axis=1)
    return (H[:, None] * X).sum(0), H[interior], L ** 3


@pytest.mark.parametrize("kind,npe", [("t4", 4), ("h8", 8)])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("st", [1.0, 1.3])
def test_tensor_conduction_first_moment(kind, npe, axis, st):
    """Uniform reference gradient G e_axis under u = (s - 1) X e_x.  Consistent loads of a uniform
    flux have first moment sum_a H_a X_a = V K0 G (linear fields are reproduced) and vanish at
    interior nodes.  By hand: the spatial gradient is F^-T G = (G_x / s, G_y, G_z), the spatial
    flux D F^-T G, and the Piola pull-back J F^-1 with J = s gives
    K0 = [[D_xx/s, D_xy, D_xz], [D_xy, s D_yy, s D_yz], [D_xz, s D_yz, s D_zz]] (Eq. 16)."""
    rng = np.random.default_rng(100 + axis)
    D = spd(rng)
    G = np.zeros(3)
    G[axis] = 400.0
    mom, Hint, V = first_moment(kind, npe, D, lambda X: X @ (np.diag([st, 1, 1]) - np.eye(3)).T, G)
    K0 = np.array([[D[0, 0] / st, D[0, 1], D[0, 2]],
                   [D[0, 1], st * D[1, 1], st * D[1, 2]],
                   [D[0, 2], st * D[1, 2], st * D[2, 2]]])
    assert np.allclose(mom, V * K0 @ G, rtol=1e-10, atol=1e-14 * V * 400.0)
    assert np.abs(Hint).max() < 1e-11 * V * 400.0 / 0.02


@pytest.mark.parametrize("kind,npe", [("t4", 4), ("h8", 8)])
def test_tensor_conduction_rigid_rotation(kind, npe):
    """Rigid rotation u = (R - I) X of a body under a fixed conductivity tensor D of Eq. 16: the
    spatial gradient is R G, the flux D R G, its pull-back R^T D R G: first moment V R^T D R G."""
    rng = np.random.default_rng(11)
    D, R = spd(rng), rotation(rng)
    G = np.array([300.0, -200.0, 100.0])
    mom, Hint, V = first_moment(kind, npe, D, lambda X: X @ (R - np.eye(3)).T, G)
    assert np.allclose(mom, V * R.T @ D @ R @ G, rtol=1e-10, atol=1e-14 * V * 400.0)
    assert np.abs(Hint).max() < 1e-11 * V * 400.0 / 0.02


@pytest.mark.parametrize("kind,npe", [("t4", 4), ("h8", 8)])
def test_tensor_conduction_special_cases(kind, npe):
    """D = k I reproduces the isotropic law and D = k I + (k_m - k) a a the transversely isotropic
    one (the tensor mode reduces to the other two)."""
    L, n = 0.02, 3
    X, conn, _ = W.box_mesh(kind, n, L)
    rng = np.random.default_rng(3)
    u = 1e-3 * np.sin(60 * X) @ rng.standard_normal((3, 3))
    T = T0 + 50.0 * np.cos(40 * X).sum(1)
    a = rng.standard_normal(3); a /= np.linalg.norm(a)
    ne = len(conn)
    for mode, k_m, D in ((0, 0.5, 0.5 * np.eye(3)), (1, 1.4, 0.5 * np.eye(3) + 0.9 * np.outer(a, a))):
        ref = oracle.OracleSim(npe, X, conn, dict(TEN, cond_mode=mode, k_m=k_m), a0=np.tile(a, (ne, 1)), dt=1e-3)
        ten = oracle.OracleSim(npe, X, conn, TEN, a0=np.tile(a, (ne, 1)), D=np.tile(D, (ne, 1, 1)), dt=1e-3)
        _, H0 = ref.loads(u, T)
        _, H1 = ten.loads(u, T)
        assert np.allclose(H1, H0, rtol=1e-11, atol=1e-12 * np.abs(H0).max())


@pytest.mark.parametrize("Tb", [300.0, 336.65, 370.0])
def test_tensor_conduction_kT(Tb):
    """With Table 5's k(T) on, the tensor scales by k(T)/k: first moment V (k(Tb)/k) D G for a
    gradient small enough that every element sees k(Tb)."""
    L, n = 0.02, 3
    X, conn, _ = W.box_mesh("h8", n, L)
    tab = W.paper_table5_material()
    p = dict(TEN, k=tab["k"], ckT_on=1, ckT_lo=tab["ckT_lo"], ckT_hi=tab["ckT_hi"], c_hi=tab["c_hi"], k_hi=tab["k_hi"])
    D = spd(np.random.default_rng(4))
    G = np.array([1e-3 / L, 0.0, 0.0])
    s = oracle.OracleSim(8, X, conn, p, D=np.tile(D, (len(conn), 1, 1)), dt=1e-3)
    _, H = s.loads(np.zeros_like(X), Tb + X @ G)
    w = min(max((Tb - 310.15) / 53.0, 0.0), 1.0)
    ratio = (0.53 + 0.22 * w) / 0.53
    assert np.allclose((H[:, None] * X).sum(0), L ** 3 * ratio * D @ G, rtol=1e-5)


def test_tensor_conduction_missing_tensor_rejected():
    X, conn, _ = W.box_mesh("t4", 1, 0.01)
    with pytest.raises(ValueError):
        oracle.OracleSim(4, X, conn, TEN, dt=1e-3)
