"""The pins must catch a plausible slip in the step they cover.  Each case
plants one mistake in a copy of the oracle source (on the CPU), builds it and
runs the pin against it: the pin has to fail.  The unaltered oracle passes the
same pins in their own test modules."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import test_oracle_deposit_launch_picard as P  # noqa: E402
import test_oracle_convergence as CV  # noqa: E402
import test_oracle_raytrace as RT  # noqa: E402
import test_oracle_pda_nl as NL  # noqa: E402
import test_oracle_raytrace_image as IM  # noqa: E402
import test_oracle_visibility as VI  # noqa: E402

SRC = os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle", "mcrt_oracle.c")

MUTANTS = {
    # the deposit loses its density factor
    "deposit_without_rho": ("  return m->rho[c] * t_interp(t, t->kbar, Tc) * ell;",
                            "  return t_interp(t, t->kbar, Tc) * ell;"),
    # the deposit takes the Rosseland extinction instead of kappa-bar
    "deposit_chi_for_kbar": ("  return m->rho[c] * t_interp(t, t->kbar, Tc) * ell;",
                             "  return m->rho[c] / (3.0 * t_interp(t, t->Drho, Tc)) * ell;"),
    # the diffusion coefficient loses its 1/3
    "deposit_D_times_3": ("  double D = t_interp(t, t->Drho, Tc) / m->rho[c];",
                          "  double D = 3.0 * t_interp(t, t->Drho, Tc) / m->rho[c];"),
    # the launch bin is shifted by one
    "launch_bin_shift": ("    while (k < nl - 1 && !(t->star_cdf[k] > xs)) ++k;",
                         "    while (k < nl - 1 && !(t->star_cdf[k + 1] > xs)) ++k;"),
    # Picard keeps D at the Monte Carlo temperature
    "picard_frozen_D": ("    rc = pda_solve_once(m, t, &g, region_out, T_out, T_mc, NULL, 1, u);",
                        "    rc = pda_solve_once(m, t, &g, region_out, T_mc, T_mc, NULL, 1, u);"),
    # the split tally takes the even-numbered packets
    "half_tally_even": ("        if (E_half && (pid & 1)) E_half[c] += eps;",
                        "        if (E_half && !(pid & 1)) E_half[c] += eps;"),
    # the spread of the halves loses its factor 2
    "conv_half_spread": ("      const double rel = (2.0 * E_half[c] - E) / E;",
                         "      const double rel = (E_half[c] - E) / E;"),
    # the slope of the inversion enters unsquared
    "conv_slope_unsquared": ("      s2 = slope * slope * rel * rel;",
                             "      s2 = slope * rel * rel;"),
    # the formal solution forgets to attenuate what lies behind
    "ray_no_attenuation": ("            I[k] = I[k] * at + S[(size_t)c * nl + k] * (1.0 - at);",
                           "            I[k] = I[k] + S[(size_t)c * nl + k] * (1.0 - at);"),
    # a ray stands for one azimuth only, not also its mirror image
    "ray_area_halved": ("      const double area = PI * (b_hi * b_hi - b_lo * b_lo) / n_phi;",
                        "      const double area = PI * (b_hi * b_hi - b_lo * b_lo) / (2 * n_phi);"),
    "ray_area_halved_thick": ("      const double area = PI * (b_hi * b_hi - b_lo * b_lo) / n_phi;",
                              "      const double area = PI * (b_hi * b_hi - b_lo * b_lo) / (2 * n_phi);"),
    # the mean intensity loses its 4 pi
    "mean_intensity_no_4pi": ("    const double iv = V[c] > 0.0 ? 1.0 / (4.0 * PI * V[c]) : 0.0;",
                              "    const double iv = V[c] > 0.0 ? 1.0 / V[c] : 0.0;"),
    # the nonlinear Jacobian drops the dependence of D on T (the linear operator)
    "nl_jacobian_without_dDdT": (
        "      dRdu[c] = -R[c] * t_slope(t, t->Drho, T) / Drho * T / (4.0 * u[c]);",
        "      dRdu[c] = 0.0;"),
    # the resistance grows where D rho grows
    "nl_dRdu_sign": (
        "      dRdu[c] = -R[c] * t_slope(t, t->Drho, T) / Drho * T / (4.0 * u[c]);",
        "      dRdu[c] = R[c] * t_slope(t, t->Drho, T) / Drho * T / (4.0 * u[c]);"),
    # the image stores the rays azimuth-major instead of ring-major
    "image_layout_swapped": (
        "          double* dst = img + (((size_t)q * (nr + 1) * n_sub + ring) * n_phi + ph) * nl;",
        "          double* dst = img + (((size_t)q * n_phi + ph) * (nr + 1) * n_sub + ring) * nl;"),
    # the image plane's first axis leaves out the tilt of the pole
    "image_axis_untilted": ("    const double e1[3] = {ci, 0.0, -si};    /* image plane */",
                            "    const double e1[3] = {0.0, 0.0, -1.0};    /* image plane */"),
    # the visibility forgets the mirror images of the rays
    "visibility_no_mirror": ("            for (int mirror = 0; mirror < 2; ++mirror) {",
                             "            for (int mirror = 0; mirror < 1; ++mirror) {"),
}

PIN = {
    "deposit_without_rho": lambda o: P.test_mrw_deposit_vs_explicit_walk(o, 10.0, 20000),
    "deposit_chi_for_kbar": lambda o: P.test_mrw_deposit_vs_explicit_walk(o, 10.0, 20000),
    "deposit_D_times_3": lambda o: P.test_mrw_deposit_vs_explicit_walk(o, 10.0, 20000),
    "launch_bin_shift": lambda o: P.test_launch_spectrum_is_stellar(o),
    "picard_frozen_D": lambda o: P.test_pda_picard_on_temperature_dependent_D(o),
    "half_tally_even": lambda o: CV.test_odd_tally_is_the_odd_packets_alone(o),
    "conv_half_spread": lambda o: CV.test_split_noise_against_run_to_run_spread(o, _passes()),
    "conv_slope_unsquared": lambda o: CV.test_split_noise_against_run_to_run_spread(o, _passes()),
    "ray_no_attenuation": lambda o: RT.test_thick_isothermal_shell(o),
    "ray_area_halved": lambda o: RT.test_thin_isothermal_shell(o),
    "ray_area_halved_thick": lambda o: RT.test_thick_isothermal_shell(o),
    "mean_intensity_no_4pi": lambda o: RT.test_mean_intensity_follows_the_dilution_law(o),
    "nl_jacobian_without_dDdT":
        lambda o: NL.test_nonlinear_gradient_matches_finite_differences(o, "logrho", True),
    "nl_dRdu_sign":
        lambda o: NL.test_nonlinear_gradient_matches_finite_differences(o, "logrho", False),
    "image_layout_swapped": lambda o: IM.test_isothermal_shell_image_is_the_chord_law(o),
    "image_axis_untilted": lambda o: IM.test_pole_on_image_is_axisymmetric(o),
    "visibility_no_mirror": lambda o: VI.test_ring_is_a_bessel_function(o),
}


def _passes():
    from multiprocessing import get_context
    with get_context("fork").Pool(8) as pool:
        return pool.map(CV._pass, [(k, 100000) for k in range(16)])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_catches_mutant(oracle_mod, tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "the mutation site moved: " + name
    path = oracle_mod.build_variant(src.replace(old, new), str(tmp_path / ("lib_%s.so" % name)))
    oracle_mod.use_library(path)
    try:
        with pytest.raises(AssertionError):
            PIN[name](oracle_mod)
    finally:
        oracle_mod.use_library(None)
