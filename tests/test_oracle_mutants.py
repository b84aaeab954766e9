"""The oracle's pins have teeth: plant one plausible mistake at a time in a
temporary copy of the oracle's C source (never in the committed file), build
it, and check that the pin suite fails on it."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hprqp_oracle.c")

MUTANTS = {
    "halpern_sign": ("const double rho = 1.0 / (double)(t + 2);\n      for (int i = 0; i < m; ++i) y[i] = rho * ya[i] + (1.0 - rho) * (2.0 * yb[i] - y[i]);",
                     "const double rho = 1.0 / (double)(t + 2);\n      for (int i = 0; i < m; ++i) y[i] = rho * ya[i] + (1.0 - rho) * (2.0 * yb[i] + y[i]);"),
    "halpern_index": ("1.0 / (double)(t + 2)", "1.0 / (double)(t + 3)"),
    "w_half_coef": ("(sQ * w[j] + xh[j]) / (1.0 + sQ)", "(sQ * w[j] + xh[j]) / (1.0 + 2.0 * sQ)"),
    "ybar_sign": ("(clamp(ry[i], P->l[i], P->u[i]) - ry[i]) / (sigma * lamA)",
                  "(ry[i] - clamp(ry[i], P->l[i], P->u[i])) / (sigma * lamA)"),
    "wbar_coef": ("sigma / (1.0 + sQ) * ATd[j]", "1.0 / (1.0 + sQ) * ATd[j]"),
    "xhat": ("xh[j] = 2.0 * xb[j] - x[j];", "xh[j] = xb[j];"),
    "rz_c_sign": ("rz[j] = x[j] + sigma * (-Qw[j] + ATy[j] - P->c[j]);",
                  "rz[j] = x[j] + sigma * (-Qw[j] + ATy[j] + P->c[j]);"),
    "v_sign": ("vv[j] = xh[j] + sigma * (Qw[j] - Qwh[j]);", "vv[j] = xh[j] + sigma * (Qwh[j] - Qw[j]);"),
    "theta1_cross": ("- 2.0 * dot(Qdw, ATdy, n);", "+ 2.0 * dot(Qdw, ATdy, n);"),
    "mnorm_sigma2": ("sigma * sigma * th[2] / (1.0 + sigma * lamQ)", "sigma * th[2] / (1.0 + sigma * lamQ)"),
    "dual_obj_sign": ("else sup += P->l[i] * y[i];", "else sup -= P->l[i] * y[i];"),
    "beta_swap": ("double beta = exp(-ratio);\n            sigma = exp(beta * log(snew) + (1.0 - beta) * log(sigma));\n          }\n          alpha3 = orc_alpha3_next(alpha3, ratio);\n          /* u^{r+1,0}",
                  "double beta = exp(-ratio);\n            sigma = exp((1.0 - beta) * log(snew) + beta * log(sigma));\n          }\n          alpha3 = orc_alpha3_next(alpha3, ratio);\n          /* u^{r+1,0}"),
    "kron_transpose": ("acc += T[i + (size_t)s * b] * B[j + (size_t)p * b];",
                       "acc += T[i + (size_t)s * b] * B[b + (size_t)p * j];"),
    "power_no_norm": ("for (int i = 0; i < k; ++i) v[i] = w[i] / nw;", "for (int i = 0; i < k; ++i) v[i] = w[i] / (2.0 * nw);"),
    "precond_box_unscaled": ("L[j] = P->L[j] / D[j]; U[j] = P->U[j] / D[j];", "L[j] = P->L[j]; U[j] = P->U[j];"),
    "precond_y_unscale": ("for (int i = 0; i < m; ++i) y_out[i] *= E[i];", "for (int i = 0; i < m; ++i) y_out[i] /= E[i];"),
    "ruiz_no_sqrt": ("if (nrm[i] > 0.0) f[i] /= sqrt(nrm[i]);", "if (nrm[i] > 0.0) f[i] /= nrm[i];"),
    "precond_stop_on_scaled": ("        if (D) {\n          for (int i = 0; i < m; ++i) dy[i] = E[i] * yb[i];\n          for (int j = 0; j < n; ++j) { dw[j]",
                               "        if (0) {\n          for (int i = 0; i < m; ++i) dy[i] = E[i] * yb[i];\n          for (int j = 0; j < n; ++j) { dw[j]"),
    "soft_threshold_sign": ("(r > t) ? r - t :", "(r > t) ? r + t :"),
    "l1_missing_in_pobj": ("double pobj = 0.5 * xQx + cx + P->l1_weight * l1;", "double pobj = 0.5 * xQx + cx;"),
    "gram_abs_values": ("acc += P->gram_val[k] * x[P->gram_col[k]];", "acc += fabs(P->gram_val[k]) * x[P->gram_col[k]];"),
    "conj_ignores_lambda": ("(isinf(L) && z > lam + slack)", "(isinf(L) && z > slack)"),
    "ruiz_col_part": ("if (p == 0) { if (a > ny[i]) ny[i] = a; if (a > na[j]) na[j] = a; }",
                      "if (p == 0) { if (a > ny[i]) ny[i] = a; }"),
}

# mistakes in the restart rule of Section 3.2, the alpha3 tightening of Section 4.1
# and the bookkeeping that feeds them, each caught by the dedicated restart pins
# alone (hand-worked cases and the replay of a traced solve)
RESTART_MUTANTS = {
    "restart_c1_strict": ("if (R <= alpha1 * Rr0) mask |= 1;", "if (R < alpha1 * Rr0) mask |= 1;"),
    "restart_c1_uses_alpha2": ("if (R <= alpha1 * Rr0) mask |= 1;", "if (R <= alpha2 * Rr0) mask |= 1;"),
    "restart_c2_strict": ("R <= alpha2 * Rr0 && R > Rprev", "R < alpha2 * Rr0 && R > Rprev"),
    "restart_c2_uses_alpha1": ("R <= alpha2 * Rr0 && R > Rprev", "R <= alpha1 * Rr0 && R > Rprev"),
    "restart_c2_ge": ("R <= alpha2 * Rr0 && R > Rprev", "R <= alpha2 * Rr0 && R >= Rprev"),
    "restart_c2_direction": ("R <= alpha2 * Rr0 && R > Rprev", "R <= alpha2 * Rr0 && R < Rprev"),
    "restart_c2_first_check": ("if (Rprev >= 0.0 && R <= alpha2", "if (R <= alpha2"),
    "restart_c3_strict": ("if ((double)t >= alpha3 * (double)k) mask |= 4;",
                          "if ((double)t > alpha3 * (double)k) mask |= 4;"),
    "alpha3_threshold_zero": ("return (ratio <= 0.1) ? 0.2 : alpha3;", "return (ratio <= 0.0) ? 0.2 : alpha3;"),
    "alpha3_strict": ("return (ratio <= 0.1) ? 0.2 : alpha3;", "return (ratio < 0.1) ? 0.2 : alpha3;"),
    "alpha3_value": ("return (ratio <= 0.1) ? 0.2 : alpha3;", "return (ratio <= 0.1) ? 0.1 : alpha3;"),
    "alpha3_not_kept": ("return (ratio <= 0.1) ? 0.2 : alpha3;", "return (ratio <= 0.1) ? 0.2 : 0.5;"),
    "restart_prev_updated_first": ("        int do_restart = 0;\n        if (!(kkt == kkt) || !(R == R)) term = ORC_NUMERICAL;        /* NaN guard */",
                                   "        int do_restart = 0; Rprev = R;\n        if (!(kkt == kkt) || !(R == R)) term = ORC_NUMERICAL;        /* NaN guard */"),
    "restart_ref_every_check": ("      t += 1; k += 1;\n      if (t == 1) Rr0 = R;",
                                "      t += 1; k += 1;\n      if (t == 1 || is_check) Rr0 = R;"),
    "restart_ref_first_check": ("      t += 1; k += 1;\n      if (t == 1) Rr0 = R;",
                                "      t += 1; k += 1;\n      if (Rr0 < 0.0 && is_check) Rr0 = R;"),
    "restart_global_t": ("do_restart = orc_restart_test(R, Rr0, Rprev, t, k,",
                         "do_restart = orc_restart_test(R, Rr0, Rprev, k, k,"),
    "restart_beta_ref_each_restart": ("          if (R0ref < 0.0) R0ref = R;\n          double ratio = R / R0ref;\n          if (opt->enable_sigma_update) {",
                                      "          R0ref = R;\n          double ratio = R / R0ref;\n          if (opt->enable_sigma_update) {"),
}

# mistakes in HPR on the primal reformulations (Appendix A), caught by its own pin file
PRIMAL_MUTANTS = {
    "p1_tau_without_lamQ": ("const double tau = lamQ + sigma * lamA;", "const double tau = sigma * lamA;"),
    "p_no_extrapolation": ("e[i] = 2.0 * yb[i] - y[i];", "e[i] = yb[i];"),
    "p_s_shift_sign": ("const double r = Ax[i] - y[i] / sigma;", "const double r = Ax[i] + y[i] / sigma;"),
    "p2_v_prox_term": ("(sigma * x[j] - t[j] + lamQ * v[j] - Qin[j]) / (lamQ + sigma)",
                       "(sigma * x[j] - t[j] - Qin[j]) / (lamQ + sigma)"),
    "p2_t_sign": ("tb[j] = t[j] + sigma * (vb[j] - x[j]);", "tb[j] = t[j] - sigma * (vb[j] - x[j]);"),
    "p2_kappa": ("const double kap = sigma * (1.0 + lamA);", "const double kap = sigma * lamA;"),
    "p_metric_cross": ("double r = -2.0 * dot(Adx, dy, m) + dot(dy, dy, m) / sigma;",
                       "double r = 2.0 * dot(Adx, dy, m) + dot(dy, dy, m) / sigma;"),
    "p2_metric_dt_cross": ("- 2.0 * dot(dx, dt, n) + dot(dt, dt, n) / sigma", "+ dot(dt, dt, n) / sigma"),
    "p2_halpern_v": ("v[j] = rho * va[j] + (1.0 - rho) * (2.0 * vb[j] - v[j]);",
                     "v[j] = rho * va[j] + (1.0 - rho) * vb[j];"),
    "p_sigma_inverted": ("double snew = sqrt(th2 / th1);", "double snew = sqrt(th1 / th2);"),
    "p_zbar_sign": ("      zb[j] = tau * (xb[j] - r);", "      zb[j] = tau * (r - xb[j]);"),
}


# mistakes in the QAP-relaxation operator (Section 4.5), caught by its pin file
QAP_MUTANTS = {
    "qap_S_sign": ("P->kron_S[i + (size_t)s * a] * x[a + (size_t)s * j];\n          out[i + (size_t)s * j] -= acc;",
                   "P->kron_S[i + (size_t)s * a] * x[a + (size_t)s * j];\n          out[i + (size_t)s * j] += acc;"),
    "qap_T_right_side": ("acc += x[i + (size_t)s * b] * P->kron_T[j + (size_t)p * b];",
                         "acc += x[b + (size_t)s * j] * P->kron_T[i + (size_t)p * b];"),
    "qap_S_dropped": ("    if (P->kron_S)\n", "    if (0)\n"),
}


@pytest.mark.parametrize("name", sorted(QAP_MUTANTS))
def test_qap_pins_catch_mutant(name, tmp_path):
    old, new = QAP_MUTANTS[name]
    _run_mutant(old, new, "test_qap.py", tmp_path, name)


@pytest.mark.parametrize("name", sorted(RESTART_MUTANTS))
def test_restart_pins_catch_mutant(name, tmp_path):
    old, new = RESTART_MUTANTS[name]
    _run_mutant(old, new, "test_oracle_pins.py", tmp_path, name, select="restart or alpha3")


def _run_mutant(old, new, pin_file, tmp_path, name, select=None):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC", "-shared",
                           "-I", os.path.join(ROOT, "oracle"), "-o", str(lib), str(msrc), "-lm"])
    env = dict(os.environ, HPRQP_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", pin_file)] + (["-k", select] if select else []),
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pin suite"
    if select:      # a pin failed, rather than no test being selected
        assert " failed" in r.stdout.strip().splitlines()[-1], r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(PRIMAL_MUTANTS))
def test_primal_pins_catch_mutant(name, tmp_path):
    old, new = PRIMAL_MUTANTS[name]
    _run_mutant(old, new, "test_oracle_primal.py", tmp_path, name)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC", "-shared",
                           "-I", os.path.join(ROOT, "oracle"), "-o", str(lib), str(msrc), "-lm"])
    env = dict(os.environ, HPRQP_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pin suite"
