"""The oracle's pins catch plausible mistakes in it.

Each case plants one mistake in a copy of the oracle's C source (a dropped
or mistyped constant, a wrong sign or index, a transposed operand, a wrong
stage node), builds it, and runs the pins that should see it on that build:
at least one must fail.  The unmodified copy passes the same pins.  Nothing
here touches the GPU path; the mutants run on the CPU only.
"""
import os
import shutil

import pytest

import test_oracle_paper_grids as PG
import test_oracle_pins as P
import test_oracle_transport as TR
import test_oracle_variants as V
import test_oracle_weno_exact as X

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


def weno_exact(orc):
    X.test_oracle_weno_b_equals_exact_rational_evaluation(orc, 1, "random")
    X.test_oracle_weno_b_equals_exact_rational_evaluation(orc, 3, "jumps")


def linear_exact(orc):
    P.test_linear_part_exact_on_gaussian(orc, 3, 0.25, 4)


# (name, text in kzk_oracle.c, replacement, which occurrence (None: all), pins)
MUTATIONS = [
    ("indicator weight 13/12 -> 1/12", "13.0 / 12.0 * sq(", "1.0 / 12.0 * sq(", None, [weno_exact]),
    ("indicator weight 1/4 -> 1/2 (beta_0)", "0.25 * sq(v[0] - 4.0 * v[1] + 3.0 * v[2])",
     "0.5 * sq(v[0] - 4.0 * v[1] + 3.0 * v[2])", None, [weno_exact]),
    ("ideal weight 6/10 -> 5/10", "double a1 = 0.6 / sq(eps + b1);", "double a1 = 0.5 / sq(eps + b1);", None,
     [weno_exact]),
    ("candidate q_2 coefficient", "double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;",
     "double q2 = (2.0 * v[2] + 4.0 * v[3] - v[4]) / 6.0;", None, [weno_exact]),
    ("F- stencil not mirrored", "vm[r] = fm[wrap(i + 3 - r, n)];   /* f- mirrored",
     "vm[r] = fm[wrap(i - 1 + r, n)];   /* f- mirrored", None, [weno_exact]),
    ("Lax-Friedrichs speed halved in f+", "fp[j] = 0.5 * (f + alpha * u[j]);",
     "fp[j] = 0.5 * (f + 0.5 * alpha * u[j]);", 0, [weno_exact]),
    ("diffraction sign", "return absorb + I * Dbar * ky * ky / (2.0 * kt);",
     "return absorb - I * Dbar * ky * ky / (2.0 * kt);", None, [linear_exact]),
    ("wavenumbers not angular", "return 2.0 * PI * (double)s / len;", "return PI * (double)s / len;", None,
     [linear_exact]),
    ("absorption sign", "double absorb = -c->A * kt * kt;", "double absorb = c->A * kt * kt;", None,
     [lambda o: P.test_absorption_mode_decays_exactly(o, 3)]),
    ("diffraction kept at the tau-Nyquist index", "if (2 * m == c->nt) return absorb;", "", None,
     [P.test_symbol_special_columns_and_hermitian_symmetry]),
    ("mean tau-mode of F(b) kept", "for (int n = 0; n < c->ny; ++n) B[(size_t)n * c->nt] = 0;", "", None,
     [P.test_mean_tau_mode_of_b_is_zeroed]),
    ("stage values transposed in the combine",
     "h * ((P1[i] - P2[i]) * w->B0[i] + P2[i] * w->B1[i])", "h * ((P1[i] - P2[i]) * w->B1[i] + P2[i] * w->B0[i])",
     None, [P.test_affine_forcing_integrated_exactly]),
    ("stage 2 uses nl(x_n)", "eval_b(c, xn1, c->nl[s + 1], w->u, w->b);", "eval_b(c, xn1, c->nl[s], w->u, w->b);",
     None, [P.test_exprk22_second_order_with_x_dependent_coefficients]),
    ("multipliers of step 0 reused", "build_mults(c, &w->M, c->Dbar[s]);", "build_mults(c, &w->M, c->Dbar[0]);", 0,
     [P.test_linear_part_exact_with_x_dependent_diffraction]),
    ("phi series factorial", "f *= (double)(j + k + 1);", "f *= (double)(j + k + 2);", None,
     [lambda o: P.test_phi_against_arbitrary_precision(o, 2)]),
    ("FFT twiddle sign", "double ang = sign * 2.0 * PI * (double)k / (double)n;",
     "double ang = -sign * 2.0 * PI * (double)k / (double)n;", None,
     [lambda o: P.test_fft_matches_direct_dft(o, 16)]),
    ("field-wide LF speed ignored", "double m = c->lf_global ? gmax : max_abs(uj, c->nt);",
     "double m = max_abs(uj, c->nt);", 0, [P.test_field_wide_lf_speed_reduces_to_heun_with_the_global_maximum]),
    ("adjoint: LF-speed term without the sign of u",
     "u_bar[(size_t)j * nt + k] += abar[j] * fabs(nl) * (uj[k] > 0 ? 1.0 : -1.0) / cnt;",
     "u_bar[(size_t)j * nt + k] += abar[j] * fabs(nl) / cnt;", None,
     [lambda o: P.test_full_adjoint_matches_central_differences(o, 3)]),
    ("adjoint: weight derivative factor", "double da = -2.0 * d[r] / pow(eps + beta[r], 3) * dbeta[r][s];",
     "double da = -1.0 * d[r] / pow(eps + beta[r], 3) * dbeta[r][s];", None,
     [P.test_weno_adjoint_matches_finite_differences]),
    ("regularised shift without 1/(4 pi)", "I * kt + c->reg_eps / (4.0 * PI)", "I * kt + c->reg_eps", None,
     [V.test_regularised_mean_column_follows_its_closed_form]),
    ("regularised diffraction sign", "return absorb - 0.5 * Dbar * ky * ky / (I * kt",
     "return absorb + 0.5 * Dbar * ky * ky / (I * kt", None,
     [V.test_regularised_equals_unregularised_on_fields_of_zero_tau_mean]),
    ("regularised multiplier zeroes the mean of F(b)", "    if (c->reg_eps > 0) return;\n", "", None,
     [V.test_regularised_multiplier_keeps_the_mean_of_b]),
    ("exponential Euler runs the second stage", "if (c->scheme == 1) {", "if (c->scheme == 2) {", None,
     [V.test_exponential_euler_first_order, V.test_exponential_euler_not_exact_for_x_dependent_forcing]),
    ("exponential Euler with phi2", "        memcpy(w->U, Us, sizeof(cplx) * N);",
     "        for (size_t i = 0; i < N; ++i) w->U[i] = E[i] * w->U[i] + h * P2[i] * w->B0[i];", None,
     [V.test_exponential_euler_exact_for_constant_forcing]),
    ("transport: axial velocity sign", "double cpar = 2.0 * PI * vel[3 * j];", "double cpar = -2.0 * PI * vel[3 * j];",
     None, [TR.test_constant_axial_velocity_translates_in_tau, TR.test_axial_transport_term_equals_exact_evaluation]),
    ("transport: LF speed along tau ignores U_par", "alpha = fmax(alpha, fabs(nl * uj[k] - cpar));",
     "alpha = fmax(alpha, fabs(nl * uj[k]));", None, [TR.test_axial_transport_term_equals_exact_evaluation]),
    ("transport: LF speed along y from U_par", "ay = fmax(ay, fabs(vel[3 * j + 1]));", "ay = fmax(ay, fabs(vel[3 * j]));",
     None, [TR.test_transverse_transport_term_equals_exact_evaluation]),
    ("transport: source sign", "/ dy + vel[3 * j + 2] * u[", "/ dy - vel[3 * j + 2] * u[", None,
     [TR.test_transport_flux_differences_telescope]),
    ("transport: y difference over dtau", "b[(size_t)j * nt + k] += -(F[j] - F[wrap(j - 1, ny)]) / dy",
     "b[(size_t)j * nt + k] += -(F[j] - F[wrap(j - 1, ny)]) / dtau", None,
     [TR.test_transport_b_converges_at_fifth_order]),
    ("velocity: atan2 arguments swapped", "double ang = atan2(y, x);", "double ang = atan2(x, y);", None,
     [TR.test_velocity_equals_cartesian_mode_sum]),
    ("velocity: amplitude without 1/N", "amp[n] = sqrt(E / (double)N) / c->vel_c0;",
     "amp[n] = sqrt(E) / c->vel_c0;", None, [TR.test_velocity_field_is_bounded_as_stated]),
    ("velocity: energy halved", "amp[n] = sqrt(E / (double)N) / c->vel_c0;",
     "amp[n] = sqrt(E / (double)(2 * N)) / c->vel_c0;", None,
     [TR.test_velocity_field_carries_the_energy_of_its_spectrum]),
    ("velocity: spectrum without its 1/8", "double E = 0.125 * sq(c->vel_sigma_u)", "double E = sq(c->vel_sigma_u)",
     None, [TR.test_velocity_field_carries_the_energy_of_its_spectrum]),
    ("velocity: mode vector not normal to K", "double U1 = -amp[n] * sin(th), U2 = amp[n] * cos(th);",
     "double U1 = amp[n] * cos(th), U2 = amp[n] * sin(th);", None, [TR.test_velocity_field_is_divergence_free]),
    ("mixed-radix FFT: odd-length sum with the wrong sign",
     "double ang = sign * 2.0 * PI * (double)(((long)j * k) % n) / (double)n;",
     "double ang = -sign * 2.0 * PI * (double)(((long)j * k) % n) / (double)n;", None,
     [lambda o: PG.test_mixed_radix_fft_matches_direct_dft(o, 56, -1)]),
    ("mixed-radix FFT: halves not recombined with twiddles",
     "cplx t = (cos(ang) + I * sin(ang)) * a[h + k];", "cplx t = a[h + k];", None,
     [lambda o: PG.test_mixed_radix_fft_matches_numpy(o, 448)]),
    ("adjoint: multiplier not conjugated", "w->W[i] = conj(M[i]) * V[i];", "w->W[i] = M[i] * V[i];", None,
     [lambda o: P.test_full_adjoint_matches_central_differences(o, 3)]),
]

ALL_PINS = sorted({id(f): f for m in MUTATIONS for f in m[4]}.items())


def _mutant(tmp_path, name, old, new, which):
    src = open(os.path.join(ORACLE_DIR, "kzk_oracle.c")).read()
    n = src.count(old)
    assert n >= 1, "mutation site not found: %s" % name
    if which is None:
        src = src.replace(old, new)
    else:
        assert which < n
        i = -1
        for _ in range(which + 1):
            i = src.index(old, i + 1)
        src = src[:i] + new + src[i + len(old):]
    d = tmp_path / "m"
    d.mkdir()
    shutil.copy(os.path.join(ORACLE_DIR, "kzk_oracle.h"), d / "kzk_oracle.h")
    (d / "kzk_oracle.c").write_text(src)
    return str(d)


def test_unmodified_copy_passes_the_pins(orc, tmp_path):
    d = _mutant(tmp_path, "none", "#include", "#include", 0)
    lib = orc.build(force=True, src=os.path.join(d, "kzk_oracle.c"), out=os.path.join(d, "liborc_copy.so"))
    with orc.using_library(lib):
        for _, pin in ALL_PINS:
            pin(orc)


@pytest.mark.parametrize("name,old,new,which,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(orc, tmp_path, name, old, new, which, pins):
    d = _mutant(tmp_path, name, old, new, which)
    lib = orc.build(force=True, src=os.path.join(d, "kzk_oracle.c"), out=os.path.join(d, "liborc_mut.so"))
    caught = []
    with orc.using_library(lib):
        for pin in pins:
            try:
                pin(orc)
            except AssertionError:
                caught.append(getattr(pin, "__name__", "pin"))
    assert caught, "no pin caught: %s" % name
