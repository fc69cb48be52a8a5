"""Planted mistakes in the oracle must be caught by the pins (CPU only).

Each case copies the oracle source, plants one plausible mistake (a dropped
term, a wrong sign, an off-by-one, a wrong tie rule, a wrong owner ...),
compiles it into a scratch directory and runs the pin checks against it in a
child process.  The case passes when some pin fails."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "potts_sign": ("if (x_in[u] != l) c++;", "if (x_in[u] == l) c++;"),
    "drop_log_sigma": ("(2.0 * sigma_in[l] * sigma_in[l]) + log(sigma_in[l]);", "(2.0 * sigma_in[l] * sigma_in[l]);"),
    "variance_factor": ("(d * d) / (2.0 * sigma_in[l] * sigma_in[l])", "(d * d) / (sigma_in[l] * sigma_in[l])"),
    "tie_highest_label": ("if (E[l] < m) { m = E[l]; a = l; }", "if (E[l] <= m) { m = E[l]; a = l; }"),
    "hood_sum_wrong_term": ("sh = sh + m;", "sh = sh + E[0];"),
    "total_not_summed": ("total = total + sh;", "total = sh;"),
    "owner_last_clique": ("if (g->owner[v] >= 0) continue;", ""),
    "hood_one_member_ring": ("for (i64 f = fb; f < fe; ++f) {", "for (i64 f = fb; f < fb + 1 && f < fe; ++f) {"),
    "hood_ring_too_deep": ("for (int depth = 1; depth <= k; ++depth) {", "for (int depth = 0; depth <= k; ++depth) {"),
    "last_rule_first_write": ("for (i64 e = 0; e < g->M; ++e) pick[g->hood_vid[e]] = e;",
                              "for (i64 e = g->M - 1; e >= 0; --e) pick[g->hood_vid[e]] = e;"),
    "min_rule_last_on_ties": ("if (pick[v] < 0 || m_elem[e] < m_elem[pick[v]]) pick[v] = e;",
                              "if (pick[v] < 0 || m_elem[e] <= m_elem[pick[v]]) pick[v] = e;"),
    "min_rule_ties_ignore_labels": ("&& a_elem[e] != a_elem[c]) tie[v] = 1;", ") tie[v] = 1;"),
    "adjacency_whole_hood": ("if (is_neighbor(g, v, g->hood_vid[o + jj])) iv_push(&al, (int)jj);",
                             "if (jj != j) iv_push(&al, (int)jj);"),
    "sample_std": ("double sigma = sqrt(ss / (double)cnt);", "double sigma = sqrt(ss / (double)(cnt > 1 ? cnt - 1 : 1));"),
    "empty_label_reset": ("if (cnt == 0) { mu_out[l] = mu_in[l]; sigma_out[l] = sigma_in[l]; continue; }",
                          "if (cnt == 0) { mu_out[l] = 0.0; sigma_out[l] = 1.0; continue; }"),
    "no_sigma_floor": ("if (sigma < sigma_min) sigma = sigma_min;", ""),
    "conv_non_strict": ("if (!(fabs(now - hist[W - w]) < tol)) return 0;", "if (!(fabs(now - hist[W - w]) <= tol)) return 0;"),
    "conv_window_short": ("for (int w = 1; w <= W; ++w)", "for (int w = 1; w < W; ++w)"),
    "replicate_label_major": ("for (int h = 0; h < H; ++h)\n    for (int l = 0; l < L; ++l)",
                              "for (int l = 0; l < L; ++l)\n    for (int h = 0; h < H; ++h)"),
    "clique_not_maximal": ("if (np == 0 && nx == 0) {", "if (nx == 0) {"),
    "clique_no_exclusion": ("    Xl[xn++] = u;\n", "\n"),
    "gap_sign": ("gap_elem[e] = second - m;", "gap_elem[e] = second + m;"),
    "mstep_old_labels": ("return or_mstep(g->n, y, L, x_out,", "return or_mstep(g->n, y, L, x_in,"),
}

RUNNER = """
import sys
sys.path.insert(0, {root!r})
import oracle
from tests import pins
lib = oracle.load({path!r})
for check in pins.ALL_CHECKS:
    try:
        check(lib)
    except AssertionError:
        print("caught by", check.__name__)
        sys.exit(3)
print("not caught")
sys.exit(0)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib),
                    str(mutant_src), "-lm"], check=True)
    r = subprocess.run([sys.executable, "-c", RUNNER.format(root=ROOT, path=str(lib))],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout}\n{r.stderr}"
