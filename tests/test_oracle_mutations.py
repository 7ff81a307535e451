"""The oracle's pins must catch plausible mistakes.

Each case copies oracle/mco.c, plants one mistake by text substitution, builds
the copy with the oracle's own flags, and runs the pin that should catch it
against the broken build (in a child pytest).  The pin must fail.  Only the
copy is changed; nothing here touches the GPU.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

from oracle import build as obuild

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CASES = [
    # (id, original text, planted mistake, pin that must fail)
    ("kahn_accept", "0.5 * (c * c + 1.0 / x)", "0.5 * (c * c + x)",
     "test_oracle_samplers.py::test_compton_angles_chi2"),
    ("kahn_branch", "(1.0 + 2.0 * alpha) / (9.0 + 2.0 * alpha)", "(1.0 + 2.0 * alpha) / (7.0 + 2.0 * alpha)",
     "test_oracle_samplers.py::test_compton_angles_chi2"),
    ("rayleigh_inverse", "(1.0 / cbrt(y) - 1.0) / b", "(1.0 / sqrt(y) - 1.0) / b",
     "test_oracle_samplers.py::test_rayleigh_angles_chi2"),
    ("rayleigh_thomson", "0.5 * (1.0 + cd * cd)", "0.5 * (1.0 + cd)",
     "test_oracle_samplers.py::test_rayleigh_angles_chi2"),
    ("last_step_unclipped", "inc = on_grid(inc * r);", "inc = on_grid(inc);",
     "test_oracle_transport.py::test_beer_lambert_slab"),
    ("midpoint_dropped", "* P->inv_h + 0.5f * G[a];\n    }\n    const double ts",
     "* P->inv_h;\n    }\n    const double ts",
     "test_oracle_transport.py::test_tiny_phantom_primary_brute_force"),
    ("type_order", "if (x < pe + coh) {", "if (x < pe + inc) {",
     "test_oracle_transport.py::test_interaction_fractions"),
    ("cone_solid_angle", "float ct = 1.0f - rng_u(r) * P->omc;",
     "float ct = 1.0f - rng_u(r) * rng_u(r) * P->omc;",
     "test_oracle_transport.py::test_source_multinomial_vacuum"),
    ("panel_axis_sign", "P->eu[0] = -sb;", "P->eu[0] = sb;",
     "test_oracle_transport.py::test_detector_pencil_rays"),
    ("philox_weyl", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;",
     "test_oracle_rng.py::test_philox_matches_rocrand"),
    ("photo_z4", "C_PE * z * z * z / (e * e * e)", "C_PE * z * z * z * z / (e * e * e)",
     "test_oracle_xs.py::test_photoelectric_form"),
    ("kn_term_sign", "(t1 + t2 - t3)", "(t1 - t2 + t3)",
     "test_oracle_xs.py::test_sigma_kn_vs_quadrature"),
    ("coh_series_term", "4.0L / (n + 3));", "4.0L / (n + 2));",
     "test_oracle_xs.py::test_coherent_vs_quadrature"),
    ("lerp_sign", "return t[j] + f * (t[j + 1] - t[j]);", "return t[j] + f * (t[j] - t[j + 1]);",
     "test_oracle_transport.py::test_beer_lambert_slab"),
    ("tally_grid", "int su = iu / (g->nu / g->snu)", "int su = iu % g->snu",
     "test_oracle_transport.py::test_scatter_binning"),
    ("rotate_azimuth_sign", "cp - uy * sp) / t", "cp + uy * sp) / t",
     "test_oracle_scatter.py::test_rotation_invariants"),
    ("rotate_polar_sign", "nz = uz * ct - (st * cp) * t;", "nz = uz * ct + (st * cp) * t;",
     "test_oracle_scatter.py::test_rotation_invariants"),
    ("interaction_at_step_start", "float sint = a0 + (float)((ts - tau) / inc * (double)len);",
     "float sint = a0;", "test_oracle_scatter.py::test_free_path_exponential"),
    ("scatter_angle_sign", "rotate(d, ct, (float)cos(phi), (float)sin(phi));",
     "rotate(d, -ct, (float)cos(phi), (float)sin(phi));",
     "test_oracle_scatter.py::test_single_scatter_brute_force"),
    ("energy_not_updated", "            e = e2;\n            mat_mu(c, e, mm);",
     "            mat_mu(c, e2, mm);", "test_oracle_scatter.py::test_single_scatter_brute_force"),
    # the point-detector estimator (eq. (3)-(5), section II-C-1)
    ("pd_cos_gamma", "* pdf) * cg) * area)", "* pdf) * 1.0) * area)",
     "test_oracle_pd.py::test_pd_vacuum_event_integral"),
    ("pd_lambda_sign", "(double)d[2] * dq[2]) / dist;", "(double)d[2] * dq[2]) / -dist;",
     "test_oracle_pd.py::test_pd_vacuum_event_integral"),
    ("pd_split_norm", "* (double)c->split);", ");",
     "test_oracle_pd.py::test_pd_vacuum_event_integral"),
    ("pd_response_at_incoming_energy", "lerp_tab(c->t_eta, c->J, e2);",
     "lerp_tab(c->t_eta, c->J, e);", "test_oracle_pd.py::test_pd_vacuum_event_integral"),
    ("pd_mu_at_incoming_energy", "mat_mu(c, e2, mm);", "mat_mu(c, e, mm);",
     "test_oracle_pd.py::test_pd_event_attenuated_integral"),
    ("pd_roulette_weight", "uniform01(w[2]) < x0 / c->rr_kev) {\n                x0 = c->rr_kev;",
     "uniform01(w[2]) < x0 / c->rr_kev) {\n                x0 = x0 * 1.0;",
     "test_oracle_pd.py::test_pd_matches_analog_expectation"),
    ("pd_rayleigh_norm", "(2.0 * (double)coh_g(", "(1.0 * (double)coh_g(",
     "test_oracle_pd.py::test_pd_pdf_rayleigh"),
    ("pd_attenuation", "const double x = x0 * exp(-tau);", "const double x = x0 * exp(-0.5 * tau);",
     "test_oracle_pd.py::test_pd_single_scatter_brute_force"),
    ("pd_mixed_rayleigh_angle", "rotate(om, ct, (float)cos(phi), (float)sin(phi));",
     "rotate(om, -ct, (float)cos(phi), (float)sin(phi));",
     "test_oracle_pd.py::test_pd_vacuum_event_integral"),
    ("pd_mixed_split_norm", "lerp_tab(c->t_eta, c->J, e) / (double)c->split;",
     "lerp_tab(c->t_eta, c->J, e);", "test_oracle_pd.py::test_pd_vacuum_event_integral"),
    # the deterministic primary of eq. (7) and the angular interpolation
    ("primary_cos_gamma", "acc += e_sum * (ax * da / r2);", "acc += e_sum * (da / r2);",
     "test_oracle_primary.py::test_primary_vacuum_solid_angles"),
    ("primary_midpoint", "((double)iu + (a + 0.5) / sub)", "((double)iu + (a + 0.0) / sub)",
     "test_oracle_primary.py::test_primary_vacuum_solid_angles"),
    ("primary_last_step", "(double)dl : (double)(L - a0);", "(double)dl : (double)dl;",
     "test_oracle_primary.py::test_primary_beer_lambert_box"),
    ("interp_neighbour", "o[p] = 0.5f * (a[p] + b[p]);", "o[p] = 0.5f * (a[p] + a[p]);",
     "test_oracle_primary.py::test_interp_angles_closed_form"),
    # binding effects: S(x,Z) as null collisions, Doppler broadening
    ("sf_power", "return 1.0 - 1.0 / (w2 * w2);", "return 1.0 - 1.0 / (w2 * w);",
     "test_oracle_binding.py::test_sf_null_fraction_and_law"),
    ("sf_momentum_transfer", "const double w = 1.0 + b * (0.5 * V * om);",
     "const double w = 1.0 + b * (V * om);",
     "test_oracle_binding.py::test_sf_null_fraction_and_law"),
    ("null_collision_scatters", "if (!real) continue;", "if (!real && 0) continue;",
     "test_oracle_binding.py::test_sf_primary_transmission"),
    ("doppler_discriminant", "tau * om * (2.0 - (t * tau) * (2.0 - om))",
     "tau * om * (1.0 - (t * tau) * (2.0 - om))",
     "test_oracle_binding.py::test_doppler_momentum_profile"),
    ("doppler_profile_power", "/ ((s2 * s2) * s2)", "/ (s2 * s2)",
     "test_oracle_binding.py::test_doppler_momentum_profile"),
    ("doppler_momentum_scale", "(cbrt((double)m[i].z_eff) / 0.885) / ALPHA_INV",
     "(cbrt((double)m[i].z_eff) / 0.5) / ALPHA_INV",
     "test_oracle_binding.py::test_doppler_momentum_profile"),
    ("pd_sf_factor", "pdf *= incoh_sf(c->rayl_b[m], t * t, 1.0 - lam);", "pdf *= 1.0 + 0.0 * t;",
     "test_oracle_binding.py::test_binding_pd_matches_analog"),
    ("pd_doppler_missing",
     "e2 = (float)((double)e * sample_doppler(&rd, c->pz_scale[m], ratio, 1.0 - lam));",
     "e2 = (float)((double)e2 + 0.0 * sample_doppler(&rd, c->pz_scale[m], ratio, 1.0 - lam));",
     "test_oracle_binding.py::test_pd_doppler_vacuum_event"),
]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="mco_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name,orig,bad,pin", CASES, ids=[c[0] for c in CASES])
def test_pin_catches_planted_mistake(workdir, name, orig, bad, pin):
    src = open(os.path.join(ROOT, "oracle", "mco.c")).read()
    assert src.count(orig) == 1, f"mutation anchor not unique/present: {orig!r}"
    d = os.path.join(workdir, name)
    os.makedirs(d, exist_ok=True)
    shutil.copy(os.path.join(ROOT, "oracle", "mco.h"), d)
    with open(os.path.join(d, "mco.c"), "w") as f:
        f.write(src.replace(orig, bad))
    lib = os.path.join(d, "libmut.so")
    subprocess.run(["gcc", *obuild.CFLAGS, "-o", lib, os.path.join(d, "mco.c"), "-lm"],
                   check=True)
    env = dict(os.environ, MCO_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, pin)], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 1 and "failed" in r.stdout, (name, r.stdout[-2000:])


RECON_CASES = [
    # (id, original text, planted mistake, pin that must fail) in oracle/recon.py
    ("ramp_odd_sign", "h[odd] = -1.0 /", "h[odd] = 1.0 /", "test_ramp_kernel_frequency_response"),
    ("fdk_distance_weight", "f += (R * R) / (L * L) * val", "f += val", "test_fdk_uniform_ball"),
    ("fdk_detector_scale", "fu = (av / s + nu * pu / 2) / pu - 0.5",
     "fu = (av + nu * pu / 2) / pu - 0.5", "test_fdk_uniform_ball"),
    ("eq8_sign", "- np.log(ip / (ip + np.asarray(is_, np.float64)))",
     "+ np.log(ip / (ip + np.asarray(is_, np.float64)))", "test_eq8_recovers_primary"),
    ("otsu_criterion", "v = w0 * w1 * (m0 - m1) ** 2", "v = w0 * (m0 - m1) ** 2",
     "test_otsu_two_modes"),
]


@pytest.mark.parametrize("name,orig,bad,pin", RECON_CASES, ids=[c[0] for c in RECON_CASES])
def test_recon_pin_catches_planted_mistake(name, orig, bad, pin):
    import types
    import test_oracle_recon as T
    src = open(os.path.join(ROOT, "oracle", "recon.py")).read()
    assert src.count(orig) == 1, f"mutation anchor not unique/present: {orig!r}"
    mod = types.ModuleType("recon_mutant")
    exec(compile(src.replace(orig, bad), "recon_mutant.py", "exec"), mod.__dict__)
    saved = T.recon
    T.recon = mod
    try:
        with pytest.raises(AssertionError):
            getattr(T, pin)()
    finally:
        T.recon = saved
