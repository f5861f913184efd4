"""Plant plausible mistakes in a copy of the oracle and check that the pin
suite catches every one (CPU only).

Each mutant is a one-line textual change of oracle/bjp_oracle.c compiled to
a temporary library; the pins (tests/test_oracle_pins.py) are run against it
in a subprocess and must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bjp_oracle.c")

MUTANTS = {
    "spmv_wrong_gather_index": ("s += val[k] * x[col[k]];", "s += val[k] * x[k % n];"),
    "dot_wrong_operand": ("for (int i = 0; i < n; ++i) s += a[i] * b[i];",
                          "for (int i = 0; i < n; ++i) s += a[i] * a[i];"),
    "extract_drops_first_column": ("if (col[k] >= s && col[k] < e)", "if (col[k] > s && col[k] < e)"),
    "offsets_short_blocks": ("int e = s + nb < n ? s + nb : n;", "int e = s + nb - 1 < n ? s + nb - 1 : n;"),
    "cholesky_sign": ("s -= a[(size_t)i * m + k] * a[(size_t)j * m + k];",
                      "s += a[(size_t)i * m + k] * a[(size_t)j * m + k];"),
    "cholesky_wrong_pivot": ("a[(size_t)i * m + j] = s / a[(size_t)j * m + j];",
                             "a[(size_t)i * m + j] = s / a[(size_t)i * m + i];"),
    "solve_transposed_operand": ("for (int k = i + 1; k < m; ++k) s -= L[(size_t)k * m + i] * z[k];",
                                 "for (int k = i + 1; k < m; ++k) s -= L[(size_t)i * m + k] * z[k];"),
    "pcg_beta_inverted": ("double beta = rho_new / rho;", "double beta = rho / rho_new;"),
    "pcg_residual_uses_p": ("for (int i = 0; i < n; ++i) r[i] -= alpha * q[i];",
                            "for (int i = 0; i < n; ++i) r[i] -= alpha * p[i];"),
    "pcg_direction_unpreconditioned": ("for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];",
                                       "for (int i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];"),
    "pcg_never_replaces": ("if (tres <= tol) break;", "break;"),
    "pcg_replacement_not_counted": ("info->replacements++;", "info->replacements += 0;"),
    "pcg_replaces_without_iterations_left": ("info->replacements >= max_replacements || k >= max_iter",
                                             "info->replacements >= max_replacements"),
    "pcg_true_residual_sign": ("for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];\n        double tres",
                               "for (int i = 0; i < n; ++i) q[i] = b[i] + q[i];\n        double tres"),
    # (dropping the beta_{j-1} u_{j-1} term is not listed: with full CGS2
    # reorthogonalisation that component is projected out anyway, so the
    # mutant is equivalent)
    "lanczos_alpha_wrong_basis": ("for (int i = 0; i < n; ++i) r[i] -= a * uj[i];",
                                  "for (int i = 0; i < n; ++i) r[i] -= a * vj[i];"),
    "lanczos_no_reorth": ("for (int pass = 0; pass < 2; ++pass) {", "for (int pass = 0; pass < 0; ++pass) {"),
    "lanczos_swapped_bases": ("for (int i = 0; i < n; ++i) { un[i] = r[i] / bj; vn[i] = z[i] / bj; }",
                              "for (int i = 0; i < n; ++i) { un[i] = z[i] / bj; vn[i] = r[i] / bj; }"),
    "lanczos_reorth_wrong_basis": ("for (int l = 0; l <= j; ++l) c[l] = orc_dot(n, V + (size_t)l * n, r);",
                                   "for (int l = 0; l <= j; ++l) c[l] = orc_dot(n, U + (size_t)l * n, r);"),
    "sturm_missing_square": ("d = alpha[i] - x - beta[i - 1] * beta[i - 1] / d;",
                             "d = alpha[i] - x - beta[i - 1] / d;"),
    "extremes_wrong_target": ("int target = which == 0 ? 1 : s;", "int target = which == 0 ? 1 : s - 1;"),
    "edge_grad_sign": ("grad[e] = -(lambda[ei[e]] - lambda[ej[e]]) * (x[ei[e]] - x[ej[e]]);",
                       "grad[e] = (lambda[ei[e]] - lambda[ej[e]]) * (x[ei[e]] - x[ej[e]]);"),
    "value_grad_transposed": ("grad[k] = -lambda[i] * x[col[k]];", "grad[k] = -lambda[col[k]] * x[i];"),
}


# pin groups (pytest -k expressions over tests/test_oracle_pins.py) that cover
# each oracle function
GROUP = {
    "spmv": "spmv or pcg_solution_vs_sparse",
    "dot": "dot_exact or pcg_single_block",
    "extract": "extract",
    "offsets": "uniform_offsets",
    "cholesky": "cholesky or factor",
    "solve": "apply_is_block_solve",
    "pcg": "pcg",
    "lanczos": "kappa or lanczos",
    "sturm": "tridiag or sturm",
    "extremes": "tridiag",
    "edge": "edge_grad",
    "value": "value_grad",
}


def _group(name):
    for key in GROUP:
        if name.startswith(key):
            return GROUP[key]
    raise KeyError(name)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib),
                           str(mutated), "-lm"])
    env = dict(os.environ, BJP_ORACLE_LIB=str(lib), OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          "-k", _group(name), os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 1, f"mutant {name} survived the pins (rc {res.returncode}):\n{res.stdout[-2000:]}"
