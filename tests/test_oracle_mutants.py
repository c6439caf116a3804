"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in a copy of the oracle's C source (on the CPU; nothing here touches
a GPU), builds it, and checks that the pin meant to catch that kind of
mistake now fails."""
import os
import tempfile

import pytest

import oracle as O
import test_oracle_closed_form as CF
import test_oracle_equal_prob as EP
import test_oracle_flip_bound as FB
import test_oracle_model as MD
import test_oracle_regression as RG
import test_oracle_rng as RN


def _brute_force_lp1():
    RG.test_lp1_fit_matches_bruteforce_least_squares(RG._lstsq, 2)


def _pure_expectation():
    CF.test_pure_expectation_fits_match_projection_of_closed_form(1, [16], 4, 20000)


MUTANTS = [
    # (name, original text, planted mistake, pin that must fail)
    ("drop the j=i driver term",
     "double SY = Sp[m] + orc_driver(P, i * dt, x, y1[m], zfit) * dt - cvi[m];",
     "double SY = Sp[m] - cvi[m];",
     CF.test_coupled_driver_matches_discrete_closed_form),
    ("driver uses y_j(X_j) instead of y_{j+1}(X_{j+1})",
     "double f0 = orc_driver(P, j * dt, x, ynext, zc[zuse]);",
     "double f0 = orc_driver(P, j * dt, x, fitted(P, G, table, j, 0, x), zc[zuse]);",
     CF.test_coupled_driver_matches_discrete_closed_form),
    ("sign of the kappa term",
     "return -P->r * y + P->kappa * sz;",
     "return -P->r * y - P->kappa * sz;",
     CF.test_coupled_driver_matches_discrete_closed_form),
    ("z response scaled by 1/sqrt(dt)",
     "double resp = (Sp[m] - cz[m]) * dWi[(int64_t)m * q + l] / dt;",
     "double resp = (Sp[m] - cz[m]) * dWi[(int64_t)m * q + l] / sqrt(dt);",
     _pure_expectation),
    ("Brownian increment scaled by dt",
     "const double dt = P->T / P->N, sdt = sqrt(dt);",
     "const double dt = P->T / P->N, sdt = dt;",
     _pure_expectation),
    ("path stops one step early",
     "for (int32_t j = i; j < P->N; ++j) {\n        for (int l = 0; l < q; ++l)",
     "for (int32_t j = i; j < P->N - 1; ++j) {\n        for (int l = 0; l < q; ++l)",
     _pure_expectation),
    ("start point uniform in the cube",
     "x[l] = stratify_one(P->mu, Fm, Fp, stream_uniform(s, l));",
     "x[l] = G->kind ? stratify_one(P->mu, Fm, Fp, stream_uniform(s, l))\n"
     "                : G->lo[l] + (c + stream_uniform(s, l)) * G->h[l];",
     lambda: RN.test_start_sampler_in_cube_ks_and_mean(21, 1.0)),
    ("Box-Muller pair reuses the cosine",
     "return (n % 2 == 0) ? rho * cos(theta) : rho * sin(theta);",
     "return (n % 2 == 0) ? rho * cos(theta) : rho * cos(theta);",
     RN.test_normals_uncorrelated_across_lags),
    ("Cholesky with a transposed operand",
     "for (int t = 0; t < c; ++t) s -= L[r * n + t] * L[c * n + t];",
     "for (int t = 0; t < c; ++t) s -= L[t * n + r] * L[c * n + t];",
     _brute_force_lp1),
    ("uncentred basis",
     "double centre = G->lo[l] + (c + 0.5) * G->h[l];",
     "double centre = G->lo[l] + c * G->h[l];",
     _brute_force_lp1),
    ("equal-probability edges at equal-size positions",
     "Fm = c / (double)G->cells[l];\n            Fp = (c + 1.0) / (double)G->cells[l];",
     "Fm = logistic_cdf(P->mu, -4.0 + 8.0 * c / G->cells[l]);\n"
     "            Fp = logistic_cdf(P->mu, -4.0 + 8.0 * (c + 1.0) / G->cells[l]);",
     lambda: EP.test_equal_probability_sampler_law(1.3, [5, 3])),
    ("equal-probability look-up mirrored",
     "return (double)G->cells[l] * logistic_cdf(G->mu, x);",
     "return (double)G->cells[l] * logistic_cdf(G->mu, -x);",
     lambda: EP.test_equal_probability_lookup_matches_strata(0.7, [4, 6])),
    ("equal-probability basis centred on the lower edge",
     "double m = logistic_quantile(G->mu, (c + 0.5) / (double)G->cells[l]);",
     "double m = logistic_quantile(G->mu, (c + 0.01) / (double)G->cells[l]);",
     lambda: EP.test_equal_probability_fits_match_projection(1, [8], 3, 20000)),
    ("logistic driver constant with the wrong sign",
     "return sz * (y - (2.0 + P->q) / (2.0 * P->q));",
     "return sz * (y + (2.0 + P->q) / (2.0 * P->q));",
     CF.test_logistic_root_readout_near_continuous_solution),
    ("Ornstein-Uhlenbeck drift with the wrong sign",
     "(P->b_lin ? P->b_lin[l] * x[l] : 0.0)",
     "(P->b_lin ? -P->b_lin[l] * x[l] : 0.0)",
     lambda: CF.test_ornstein_uhlenbeck_fits_match_projection_of_closed_form(1, [16], 4, 20000, [0.3], [-0.8])),
    ("state-dependent diffusion reads the first coordinate",
     "if (P->sigma_lin) diff += P->sigma_lin[l] * x[l] * dW[l];",
     "if (P->sigma_lin) diff += P->sigma_lin[l] * x[0] * dW[l];",
     lambda: CF.test_state_dependent_diffusion_fits_match_projection_of_closed_form(2, [4, 4], 12000,
                                                                                    [0.5, -0.8])),
    ("state-dependent diffusion on the wrong increment",
     "if (P->sigma_lin) diff += P->sigma_lin[l] * x[l] * dW[l];",
     "if (P->sigma_lin) diff += P->sigma_lin[l] * x[l] * dW[d - 1 - l];",
     lambda: CF.test_state_dependent_diffusion_fits_match_projection_of_closed_form(2, [4, 4], 12000,
                                                                                    [0.5, -0.8])),
    ("face-flip bound of z without the 1/dt of its response",
     "double dr = (flip[3 * m] + dcz[m]) * fabs(dWi[(int64_t)m * q + l]) / dt;",
     "double dr = (flip[3 * m] + dcz[m]) * fabs(dWi[(int64_t)m * q + l]);",
     lambda: FB.test_flip_bound_holds_against_forced_flips(*FB.CASES[0])),
    ("face-flip bound of a path without the dt of its driver terms",
     "if (flip) dS += driver_spread(P, j * dt, x, nyc, yc, nzc, zc, f0) * dt + dcv;",
     "if (flip) dS += driver_spread(P, j * dt, x, nyc, yc, nzc, zc, f0) + dcv;",
     lambda: FB.test_flip_bound_holds_against_forced_flips(*FB.CASES[0])),
    ("network flip bound skips the second hidden layer",
     "for (int layer = 1; layer <= 2; ++layer)",
     "for (int layer = 1; layer <= 1; ++layer)",
     lambda: FB.test_flip_bound_covers_bfloat16_roundings_of_the_network(*FB.NET_CASES[0])),
    ("model drift taken at t_{j+1}",
     "P->model->b(j * dt, x, P->model->params, bj);",
     "P->model->b((j + 1) * dt, x, P->model->params, bj);",
     lambda: MD.test_time_dependent_model_fits_match_projection_of_closed_form(1, [16], 4, 20000)),
    ("driver of the y response taken at t_{i+1}",
     "double SY = Sp[m] + orc_driver(P, i * dt, x, y1[m], zfit) * dt - cvi[m];",
     "double SY = Sp[m] + orc_driver(P, (i + 1) * dt, x, y1[m], zfit) * dt - cvi[m];",
     lambda: MD.test_time_dependent_model_fits_match_projection_of_closed_form(1, [16], 4, 20000)),
    ("model diffusion 5 % too large",
     "P->model->sigma_dw(j * dt, x, dW, P->model->params, sj);",
     "P->model->sigma_dw(j * dt, x, dW, P->model->params, sj);\n            for (int l = 0; l < d; ++l) sj[l] *= 1.05;",
     lambda: MD.test_time_dependent_model_fits_match_projection_of_closed_form(1, [16], 4, 20000)),
    ("singular fallback divides by M - 1",
     "beta[0] = rhs[0] / M;\n    }\n    for (int a = 0; a < nb; ++a) rec[a] = beta[a];",
     "beta[0] = rhs[0] / (M - 1);\n    }\n    for (int a = 0; a < nb; ++a) rec[a] = beta[a];",
     lambda: FB.test_singular_gram_takes_the_lp0_mean(O.LP1, O.DRV_LOGISTIC)),
    ("Philox key bump skipped",
     "k0 += weyl0;",
     "k0 += 0u;",
     RN.test_philox_matches_rocrand_engine),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(name, old, new, pin):
    with open(O._SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = O.compile_source(path, os.path.join(tmp, "libmutant.so"))
        with O.using_library(lib):
            with pytest.raises(AssertionError):
                pin()
