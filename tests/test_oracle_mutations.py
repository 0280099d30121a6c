"""The pins catch plausible mistakes in the oracle's laws.

Each case plants one mistake in a copy of the oracle's C source (a flipped sign,
a wrong end point or ramp width, the wrong modulus scaled, swapped directions,
a dropped term), compiles the copy with gcc into a temporary directory, routes
the oracle binding through it, and checks that every pin named for the case now
fails.  A control build of the unmodified source passes the same pins, so a
failure is the planted mistake's doing and not the harness's.  Everything runs
on the CPU; the committed oracle is never modified.
"""
import os

import pytest

import oracle
import test_oracle_dose_pins as D
import test_oracle_law_pins as P
import test_oracle_ortho_pins as R
import test_oracle_pins as Q

MUTATIONS = [
    # (id, text in tled_oracle.c, planted replacement, pins that must fail)
    ("muT_drop_sign",
     "return 1.0 - m->muT_drop * clamp01(", "return 1.0 + m->muT_drop * clamp01(",
     [lambda: P.test_mu_of_T_uniaxial(340.0, 1.1), P.test_mu_of_T_values]),
    ("muT_scales_kappa",
     "eta = m->eta * s, kappa = m->kappa;", "eta = m->eta * s, kappa = m->kappa * s;",
     [lambda: P.test_mu_of_T_uniaxial(340.0, 1.1), P.test_mu_of_T_with_expansion]),
    ("muT_eta_unscaled",
     "eta = m->eta * s, kappa", "eta = m->eta, kappa",
     [lambda: P.test_mu_of_T_uniaxial(340.0, 1.1)]),
    ("muT_ramp_width",
     "clamp01((T - m->muT_lo) / (m->muT_hi - m->muT_lo))",
     "clamp01(2.0 * (T - m->muT_lo) / (m->muT_hi - m->muT_lo))",
     [lambda: P.test_mu_of_T_uniaxial(325.0, 0.9), P.test_mu_of_T_values]),
    ("shrink_sign",
     "double s = 1.0 + m->shrink_eps * clamp01(", "double s = 1.0 - m->shrink_eps * clamp01(",
     [lambda: P.test_shrinkage_free_expansion(4, 330.0), lambda: P.test_shrinkage_clamped_heating(340.0, 1559.6815)]),
    ("shrink_width",
     "(Te - m->shrink_T) / m->shrink_width", "(Te - m->shrink_T) / (2.0 * m->shrink_width)",
     [lambda: P.test_shrinkage_free_expansion(8, 325.5), lambda: P.test_shrinkage_clamped_heating(325.5, 739.5914)]),
    ("shrink_onset",
     "(Te - m->shrink_T) / m->shrink_width", "(Te - m->shrink_T + 2.0) / m->shrink_width",
     [lambda: P.test_shrinkage_clamped_heating(325.5, 739.5914), lambda: P.test_shrinkage_free_expansion(4, 325.5)]),
    ("ti_expansion_swapped_axes",
     "Fth[i] = li * I3[i] + (lm - li) * A0[i] + (ln - li) * N0[i];",
     "Fth[i] = lm * I3[i] + (li - lm) * A0[i] + (ln - li) * N0[i];",
     [lambda: P.test_ti_expansion_free(4, 0), lambda: P.test_ti_expansion_clamped_heating(10.0)]),
    ("ti_expansion_fibre_ignored",
     "double b = (m->expan_mode == 1 || m->expan_mode == 2) ? 1.0 + m->alpha_m * dT : a;", "double b = a;",
     [lambda: P.test_ti_expansion_free(8, 1), lambda: P.test_ti_expansion_clamped_heating(30.0)]),
    ("ti_conduction_swapped_k",
     "D[3 * i + j] += (kmT - kT) *", "D[3 * i + j] += (kT - kmT) *",
     [lambda: P.test_ti_conduction_patch("t4", 4, (1, 0, 0), "k_m", 1.0),
      lambda: P.test_ti_conduction_oblique_first_moment("h8", 8, 0.3)]),
    ("ti_conduction_transposed_fibre",
     "(a[i] / an) * (a[j] / an);", "(a[i] / an) * (a[(j + 1) % 3] / an);",
     [lambda: P.test_ti_conduction_oblique_first_moment("t4", 4, 1.1)]),
    ("ct_reversed",
     "return m->c + w * (m->c_hi - m->c);", "return m->c_hi + w * (m->c - m->c_hi);",
     [lambda: P.test_ct_per_step_rise(336.65 + 10), lambda: P.test_ct_per_step_rise(380.0)]),
    ("ct_evaluated_at_T0",
     "double Ca = s->m.rho * heat_capacity(&s->m, T[a]) * s->Vl[a];",
     "double Ca = s->m.rho * heat_capacity(&s->m, s->m.T0) * s->Vl[a];",
     [lambda: P.test_ct_per_step_rise(350.0)]),
    ("kt_wrong_normalisation",
     "return (m->k + w * (m->k_hi - m->k)) / m->k;", "return (m->k + w * (m->k_hi - m->k)) / m->k_hi;",
     [lambda: P.test_kt_patch(336.65, 1e-5), lambda: P.test_kt_patch(300.0, 1e-10)]),
    ("metabolic_sign",
     "+ s->Qm[a] + src * s->Qr[a]", "- s->Qm[a] + src * s->Qr[a]",
     [lambda: P.test_pennes_0d_metabolic_arterial(309.0), P.test_pennes_metabolic_only_rise]),
    ("arterial_is_T0",
     "(T[a] - s->m.T_art)", "(T[a] - s->m.T0)",
     [lambda: P.test_pennes_0d_metabolic_arterial(309.0)]),
    ("ortho_n_ratio_from_alpha_m",
     "double c = (m->expan_mode == 2) ? 1.0 + m->alpha_n * dT : a;",
     "double c = (m->expan_mode == 2) ? 1.0 + m->alpha_m * dT : a;",
     [lambda: R.test_ortho_expansion_free(4, 0), R.test_ortho_clamped_heating_values]),
    ("ortho_n_not_orthogonalised",
     "double w[3] = {n_in[0] - d * mv[0], n_in[1] - d * mv[1], n_in[2] - d * mv[2]};",
     "double w[3] = {n_in[0], n_in[1], n_in[2]};",
     [lambda: R.test_ortho_expansion_free(8, 1)]),
    ("ortho_n_term_dropped",
     "+ (lm - li) * A0[i] + (ln - li) * N0[i];", "+ (lm - li) * A0[i];",
     [lambda: R.test_ortho_expansion_free(4, 2), R.test_ortho_clamped_heating_values,
      lambda: R.test_ortho_clamped_volumetric(0)]),
    ("tensor_xy_xz_swapped",
     "static const int comp[9] = {0, 3, 5, 3, 1, 4, 5, 4, 2};",
     "static const int comp[9] = {0, 5, 3, 5, 1, 4, 3, 4, 2};",
     [lambda: R.test_tensor_conduction_first_moment("t4", 4, 0, 1.3),
      lambda: R.test_tensor_conduction_rigid_rotation("h8", 8)]),
    ("tensor_kT_unscaled",
     "double ks = conductivity_scale(m, Te);", "double ks = 1.0;",
     [lambda: R.test_tensor_conduction_kT(336.65), lambda: R.test_tensor_conduction_kT(370.0)]),
    ("cem43_R_swapped",
     "double R = Tc >= 43.0 ? 0.5 : 0.25;", "double R = Tc >= 43.0 ? 0.25 : 0.5;",
     [lambda: D.test_cem43_doubles_per_kelvin_above_and_quarters_below(3, 8.0),
      lambda: D.test_cem43_doubles_per_kelvin_above_and_quarters_below(-2, 1.0 / 16)]),
    ("cem43_in_seconds",
     "cem43[a] += dt / 60.0 * pow(R, 43.0 - Tc);", "cem43[a] += dt * pow(R, 43.0 - Tc);",
     [D.test_cem43_at_43C_counts_minutes, D.test_dose_over_a_time_loop_at_held_temperatures]),
    ("cem43_sign_of_exponent",
     "pow(R, 43.0 - Tc)", "pow(R, Tc - 43.0)",
     [lambda: D.test_cem43_doubles_per_kelvin_above_and_quarters_below(1, 2.0)]),
    ("arrhenius_in_celsius",
     "exp(-Ea / (R_gas * T[a]))", "exp(-Ea / (R_gas * Tc))",
     [D.test_arrhenius_rate_set_to_one_per_second]),
    ("arrhenius_without_dt",
     "omega[a] += dt * A * exp(", "omega[a] += A * exp(",
     [D.test_arrhenius_rate_set_to_one_per_second]),
    # a few of the older pins, for the laws they pin
    ("pullback_missing_det",
     "for (int i = 0; i < 9; ++i) S0[i] = detFth * T2[i];", "for (int i = 0; i < 9; ++i) S0[i] = T2[i];",
     [lambda: Q.test_uniaxial_with_thermal_pullback(40.0), Q.test_clamped_uniform_heating]),
    ("conduction_sign",
     "double Tnew = T[a] + dt / Ca * (-Hc[a]", "double Tnew = T[a] + dt / Ca * (Hc[a]",
     [Q.test_transient_conduction_converges_to_linear_profile]),
    # the critical step (a reading): stable, and not needlessly small
    ("critical_step_without_fibre",
     "double cd = sqrt((m->kappa + 4.0 * m->mu / 3.0 + 4.0 * m->eta) / m->rho);",
     "double cd = sqrt((m->kappa + 4.0 * m->mu / 3.0) / m->rho);",
     [lambda: Q.test_critical_step_is_stable(4, 0.0)]),
    ("critical_length_t4_without_three",
     "return 3.0 * V0 / amax;", "return V0 / amax;",
     [lambda: Q.test_critical_step_is_stable(4, 0.0)]),
    # the H8 hourglass term (its coefficient is a reading; its arithmetic is pinned)
    ("hourglass_coefficient_without_eighth",
     "V0 * s / 8.0;", "V0 * s;",
     [lambda: Q.test_hourglass_closed_form_on_a_cube(0.004)]),
    ("hourglass_modulus_without_shear",
     "khg = m->hg_coef * (m->kappa + 4.0 * m->mu / 3.0) * V0", "khg = m->hg_coef * m->kappa * V0",
     [lambda: Q.test_hourglass_closed_form_on_a_cube(0.01)]),
    ("hourglass_projection_sign",
     "gam[8 * al + a] = h[al][a] - s;", "gam[8 * al + a] = h[al][a] + s;",
     [Q.test_hourglass_vanishes_on_affine_fields]),
    ("hourglass_energy_halved_twice",
     "e_hg += 0.5 * khg *", "e_hg += 0.25 * khg *",
     [lambda: Q.test_hourglass_closed_form_on_a_cube(0.004)]),
]


@pytest.fixture(scope="module")
def source():
    with open(os.path.join(os.path.dirname(oracle.__file__), "tled_oracle.c")) as f:
        return f.read()


def _outcomes(checks):
    out = []
    for chk in checks:
        try:
            chk()
        except AssertionError:
            out.append(False)
        else:
            out.append(True)
    return out


def test_control_build_passes(source, tmp_path):
    """The unmodified source, built the same way, passes every pin used below."""
    so = oracle.build_variant(source, str(tmp_path), "control")
    with oracle.using_library(so):
        for _, _, _, checks in MUTATIONS:
            assert all(_outcomes(checks))


@pytest.mark.parametrize("name,old,new,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(source, tmp_path, name, old, new, checks):
    assert source.count(old) == 1, f"mutation site of {name} not found exactly once"
    so = oracle.build_variant(source.replace(old, new), str(tmp_path), name)
    with oracle.using_library(so):
        passed = _outcomes(checks)
    assert not any(passed), f"{name}: pins that did not catch it: {[i for i, p in enumerate(passed) if p]}"
