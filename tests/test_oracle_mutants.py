"""Sensitivity of the pins: copies of the oracle with one planted mistake
each (a flipped sign, a dropped term, a wrong index, a transposed operand,
an off-by-one) are compiled on the CPU, and every copy must fail at least
one pin.  The real oracle is never modified."""
import os
import subprocess

import pytest

import oracle
import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "sf_oracle.c")

MUTANTS = {
    "trsv_sign": ("if (j < i) s -= v[p] * x[j];", "if (j < i) s += v[p] * x[j];"),
    "trsv_drop_first": ("if (j < i) s -= v[p] * x[j];", "if (j < i && p > rp[i]) s -= v[p] * x[j];"),
    "spmv_index": ("for (int p = rp[i]; p < rp[i + 1]; ++p) s += v[p] * x[ci[p]];",
                   "for (int p = rp[i]; p < rp[i + 1]; ++p) s += v[p] * x[i];"),
    "ic0_operand": ("if (ki == kj) { s -= l[pi] * l[pj];", "if (ki == kj) { s -= l[pi] * l[pi];"),
    "ic0_no_scale": ("l[p] = s / djj;", "l[p] = s;"),
    "ic0_diag_sign": ("if (ci[p] < i) d -= l[p] * l[p];", "if (ci[p] < i) d += l[p] * l[p];"),
    "ic0_last_failure": ("if (!(d > 0.0) && fail < 0) fail = i;", "if (!(d > 0.0)) fail = i;"),
    "upper_unpermuted": ("if (j > i) s -= v[perm[q]] * lam[j];", "if (j > i) s -= v[q] * lam[j];"),
    "spmv_t_unpermuted": ("s += v[perm[q]] * g[tci[q]];", "s += v[q] * g[tci[q]];"),
    "grad_transposed": ("grad_l[p] = -grad_b[i] * x[lci[p]];", "grad_l[p] = -grad_b[lci[p]] * x[i];"),
    "grad_sign": ("grad_l[p] = -grad_b[i] * x[lci[p]];", "grad_l[p] = grad_b[i] * x[lci[p]];"),
    "levels_off_by_one": ("if (j < i && level[j] + 1 > lv) lv = level[j] + 1;",
                          "if (j < i && level[j] > lv) lv = level[j];"),
    "rlevels_constant": ("if (j > i && rlev[j] + 1 > lv) lv = rlev[j] + 1;",
                         "if (j > i && rlev[j] + 1 > lv) lv = rlev[j] + 2;"),
    "ready_off_by_one": ("if (level[aci[p]] + 1 > lv) lv = level[aci[p]] + 1;",
                         "if (level[aci[p]] > lv) lv = level[aci[p]];"),
    "order_kinds_swapped": (
        "    for (int i = 0; i < n; ++i) if (level[i] == lv) order[pos++] = i;\n"
        "    for (int r = 0; r < m; ++r) if (ready[r] == lv) order[pos++] = n + r;",
        "    for (int r = 0; r < m; ++r) if (ready[r] == lv) order[pos++] = n + r;\n"
        "    for (int i = 0; i < n; ++i) if (level[i] == lv) order[pos++] = i;"),
    "validate_nonstrict": ("int ok = item[j] < item[i] ||", "int ok = item[j] <= item[i] ||"),
    "static_any_w": ("(sof[u] < sof[v] || (wof[u] == wof[v] && pos[u] < pos[v]))",
                     "(sof[u] < sof[v] || (sof[u] == sof[v] && pos[u] < pos[v]))"),
    "static_nonstrict_s": ("(sof[u] < sof[v] || (wof[u] == wof[v] && pos[u] < pos[v]))",
                           "(sof[u] <= sof[v] || (wof[u] == wof[v] && pos[u] < pos[v]))"),
    "reuse_dropped_term": ("double kl = (double)nnz_l + (double)n + (double)n;",
                           "double kl = (double)nnz_l + (double)n;"),
    "ilu0_no_divide": ("lu[p] = lu[p] / ukk;", "lu[p] = lu[p];"),
    "ilu0_sign": ("if (ji == jk) { lu[pi] -= lu[p] * lu[pk];", "if (ji == jk) { lu[pi] += lu[p] * lu[pk];"),
    "ilu0_wrong_operand": ("if (ji == jk) { lu[pi] -= lu[p] * lu[pk];", "if (ji == jk) { lu[pi] -= lu[p] * lu[pi];"),
    "ilu0_last_failure": ("if (!(d != 0.0) && fail < 0) fail = i;", "if (!(d != 0.0)) fail = i;"),
    "check_lower_upper_off_by_one": ("      if (j > i) return ORC_NOT_LOWER;", "      if (j > i + 1) return ORC_NOT_LOWER;"),
    "check_lower_no_diag_test": ("    if (!has_diag) return ORC_NO_DIAG;", "    (void)has_diag;"),
    "check_csr_range": ("if (j < 0 || j >= ncols) return ORC_BAD_CSR;", "if (j < 0 || j > ncols) return ORC_BAD_CSR;"),
    "check_csr_accepts_duplicates": (
        "if (j < 0 || j >= ncols) return ORC_BAD_CSR;\n      if (p > rp[i] && ci[p - 1] >= j)",
        "if (j < 0 || j >= ncols) return ORC_BAD_CSR;\n      if (p > rp[i] && ci[p - 1] > j)"),
    "factor_solve_intra_factor": ("if (!(item[j] < item[i])) { rc = 4; break; }",
                                  "if (!(item[j] <= item[i])) { rc = 4; break; }"),
    "factor_solve_no_solve_edge": ("if (!(item[n + j] < item[n + i])) { rc = 5; break; }", ""),
    "factor_solve_no_f_edge": ("(item[i] == item[n + i] && pos[i] < pos[n + i])", "(item[i] == item[n + i])"),
    "refine_residual_sign": ("        r[i] = b[i] - acc;", "        r[i] = b[i] + acc;"),
    "refine_no_update": ("      x[i] = (t == 0 ? 0.0 : x[i]) + (double)v[i];", "      x[i] = (t == 0 ? (double)v[i] : x[i]);"),
    "refine_residual_fp32_values": ("for (int p = rp[i]; p < rp[i + 1]; ++p) acc += l64[p] * x[ci[p]];\n        r[i]",
                                    "for (int p = rp[i]; p < rp[i + 1]; ++p) acc += (double)l32[p] * x[ci[p]];\n        r[i]"),
    "refine_sum_sign": ("          sum = sum + prod;", "          sum = sum - prod;"),
    "refine_no_divide": ("      v[i] = top / dg;", "      v[i] = top;"),
    "refine_relres_wrong_norm": ("    if (fabs(b[i]) > bmax) bmax = fabs(b[i]);", "    bmax += fabs(b[i]);"),
    "unit_lower_divides": ("      if (ci[p] < i) s -= v[p] * y[ci[p]];\n    y[i] = s;",
                           "      if (ci[p] < i) s -= v[p] * y[ci[p]];\n    y[i] = s / 7.0;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found uniquely: " + name
    path = tmp_path / ("m_%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("m_%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so),
                           str(path), "-lm"])
    orc = oracle.Oracle(str(so))
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(orc)
        except AssertionError:
            failed.append(pin.__name__)
        except (ValueError, IndexError, FloatingPointError):
            failed.append(pin.__name__)
    assert failed, "planted mistake %s passes every pin" % name
