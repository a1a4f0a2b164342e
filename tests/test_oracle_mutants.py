"""Plant mistakes in a copy of the oracle and check that the pins catch them.

Each mutant is a one-line textual change of oracle/bhpp_oracle.c compiled into
a temporary shared object; the real oracle is untouched. A mutant counts as
caught when at least one core pin fails (or the run errors or times out).
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bhpp_oracle.c")

MUTANTS = {
    "push_drops_decay": ("(1.0 - alpha) * g->w_u[q] / g->ws_v[v] * rx", "g->w_u[q] / g->ws_v[v] * rx"),
    "push_wrong_degree": ("g->w_v[q] / g->ws_u[y] * rv", "g->w_v[q] / g->ws_v[v] * rv"),
    "t_rounds_down": ("double tr = ceil(", "double tr = floor("),
    "pi_threshold_inverted": ("wsu / g->ws_u[x] * eps_f / lambda", "g->ws_u[x] / wsu * eps_f / lambda"),
    "combine_wrong": ("beta[x] = pif[x] + w.pib[x]", "beta[x] = pif[x] + pif[x]"),
    "fppr_not_converted": ("pif[x] = g->ws_u[x] / wsu * w.pib[x]", "pif[x] = w.pib[x]"),
    "powiter_no_alpha": ("out[x] = alpha * pi[x]", "out[x] = pi[x]"),
    "lambda_no_slack": ("double a = rmax + (double)g->nu * pow(1.0 - alpha, (double)tau + 1.0);",
                        "double a = rmax;"),
    "gamma_backward_mass": ("gamma += g->ws_u[x] / wsu * w.r[x]", "gamma += w.r[x]"),
    "forward_series_transposed": ("        row_times_P(g, p, tv, nx);\n        double* t = p;",
                                  "        P_times_col(g, p, tv, nx);\n        double* t = p;"),
    "ws_is_degree": ("for (int64_t p = g->rp_u[x]; p < g->rp_u[x + 1]; ++p) s += g->w_u[p];",
                     "for (int64_t p = g->rp_u[x]; p < g->rp_u[x + 1]; ++p) s += 1.0;"),
    "ss_threshold_eps": ("w.thr[x] = eps_b;", "w.thr[x] = eps;"),
    "warm_residue_sign": ("r_out[x] = (x == u ? 1.0 : 0.0) - (y[x]", "r_out[x] = (x == u ? 1.0 : 0.0) + (y[x]"),
    "warm_residue_no_decay": ("(y[x] - (1.0 - alpha) * py[x]) / alpha", "(y[x] - py[x]) / alpha"),
    "warm_push_positive_only": ("if (!(fabs(rx) > w->thr[x])) continue;", "if (!(rx > w->thr[x])) continue;"),
    "warm_combine_start": ("beta[x] = pif[x] + pib_ss[x]", "beta[x] = pif[x] + y0[x]"),
    "warm_fallback_never": ("if (!(info.res_l1 < 1.0 && info.res_max < 1.0)) {", "if (0) {"),
    "no_sequential_pushes": ("if (!(rmax > eps_b && rsum > eps_b)) break;", "break;"),
    "pisp_t_full_eps": ("s.t = orc_t(1.0, 0.5 * eps, alpha);", "s.t = orc_t(1.0, eps, alpha);"),
    "pisp_eps_b_full_eps": ("rc = selective_push(g, u, alpha, 0.5 * eps, pib, &s.sp_iters, &s.np);",
                            "rc = selective_push(g, u, alpha, eps, pib, &s.sp_iters, &s.np);"),
    "pisp_one_push_only": ("        if (!(rmax > thr_b)) break;\n", "        break;\n"),
    "mc_stop_inverted": ("if ((double)a[0] < stop_thr) break;", "if ((double)a[0] >= stop_thr) break;"),
    "mc_alias_coin_inverted": ("(double)rc * 0x1.0p-32 < prob[b + slot] ? slot", "(double)rc * 0x1.0p-32 >= prob[b + slot] ? slot"),
    "mc_walks_half": ("return (int64_t)ceil(2.0 * (1.0 + eps_f / 3.0)", "return (int64_t)ceil(1.0 * (1.0 + eps_f / 3.0)"),
    "alias_no_carry": ("q[l] = (q[l] + q[a]) - 1.0;", "q[l] = q[l] - 1.0;"),
    "philox_no_key_bump": ("if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }", "if (r < 0) { k0 += 0x9E3779B9u; }"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    # a formula written in both the cold and the warm path is mutated in both
    assert src.count(old) >= 1, f"mutation site for {name} missing"
    mfile = tmp_path / "mutant.c"
    mfile.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(mfile), "-lm"])
    try:
        r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "pins_lib.py"), str(lib), "stop"],
                           capture_output=True, text=True, timeout=120,
                           env=dict(os.environ, PYTHONPATH=ROOT))
    except subprocess.TimeoutExpired:
        return  # a hanging mutant is caught too
    if r.returncode != 0:
        return  # crashed: caught
    res = json.loads(r.stdout.strip().splitlines()[-1])
    assert res["failures"] > 0, f"mutant {name} passed every pin"


def test_unmutated_oracle_passes(tmp_path):
    lib = tmp_path / "liborig.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), SRC, "-lm"])
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "pins_lib.py"), str(lib)],
                       capture_output=True, text=True, timeout=120, env=dict(os.environ, PYTHONPATH=ROOT))
    assert r.returncode == 0, r.stderr
    assert json.loads(r.stdout.strip().splitlines()[-1])["failures"] == 0
