"""The CPU oracle against closed forms, exact arithmetic and hand-worked
examples (no GPU involved), and proof that those pins catch plausible
mistakes: altered copies of the oracle source must each fail a pin."""
import os
import re
import subprocess
import sys

import pytest

import oracle
import pins

ORACLE_SRC = os.path.join(os.path.dirname(oracle.__file__), "spmv_oracle.c")


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(check):
    check(oracle.default())


def _function_span(src: str, name: str):
    m = re.search(r"^(void|int) %s\(" % re.escape(name), src, flags=re.M)
    assert m, name
    start = m.start()
    nxt = re.search(r"^(void|int|/\*) ", src[m.end():], flags=re.M)
    end = m.end() + nxt.start() if nxt else len(src)
    return start, end


def _mutate(src: str, edits):
    for func, old, new in edits:
        a, b = _function_span(src, func)
        body = src[a:b]
        assert old in body, (func, old)
        src = src[:a] + body.replace(old, new, 1) + src[b:]
    return src


TRANSPOSED = """void oracle_spmv(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                 const double *val, int32_t base, const double *B, double *C)
{
    for (int64_t i = 0; i < n_rows; ++i)
        for (int64_t j = (int64_t)row_ptr[i] - base; j < (int64_t)row_ptr[i + 1] - base; ++j) {
            int64_t c = (int64_t)col_idx[j] - base;
            if (c < n_rows)
                C[c] = C[c] + val[j] * B[i];
        }
}
"""

MUTANTS = {
    "sign": [("oracle_spmv", "c = c + prod;", "c = c - prod;")],
    "dropped_last_term": [("oracle_spmv", "j < end;", "j < end - 1;")],
    "c0_ignored": [("oracle_spmv", "double c = C[i];", "double c = 0.0;")],
    "index_base_row_ptr": [("oracle_spmv", "int64_t begin = (int64_t)row_ptr[i] - base;",
                            "int64_t begin = (int64_t)row_ptr[i];")],
    "rows_wrong_index": [("oracle_spmv_rows", "int64_t i = rows[s];", "int64_t i = s;")],
    "block_column_major": [("oracle_spmv_block", "B[((int64_t)col_idx[j] - base) * ldb + t]",
                            "B[((int64_t)col_idx[j] - base) + t * ldb]")],
    "abs_missing_fabs": [("oracle_abs_spmv", "fabs(val[j]) * ", "val[j] * ")],
    "abs_c0_ignored": [("oracle_abs_spmv", "double d = fabs(C0[i]);", "double d = 0.0;")],
    "block_c0_ignored": [("oracle_spmv_block", "double c = C[i * ldc + t];", "double c = 0.0;")],
    "split_nonlocal_sign": [("oracle_spmv_split", "c = c + prod;", "c = c - prod;")],
    "split_boundary": [("oracle_split_count", "- base < h)", "- base <= h)"),
                       ("oracle_split_fill", "if (c < h)", "if (c <= h)")],
    "split_row_id": [("oracle_split_fill", "nl_rows[r] = (int32_t)i;", "nl_rows[r] = (int32_t)(i + 1);")],
    "split_drop_last_nl_row": [("oracle_spmv_split", "r < n_nl_rows;", "r < n_nl_rows - 1;")],
    "send_boundary": [("oracle_send_list_symmetric", "- base >= h)", "- base > h)")],
    "send_row_limit": [("oracle_send_list_symmetric", "i < n_rows && i < h;", "i < n_rows && i <= h;")],
    "send_any_vs_all": [("oracle_send_list_symmetric", "needed = 1;", "needed = needed + 1;"),
                        ("oracle_send_list_symmetric", "if (needed)", "if (needed == 1)")],
    "pack_reversed": [("oracle_pack", "out[k] = B[idx[k]];", "out[k] = B[idx[n - 1 - k]];")],
    "kpm_no_factor_two": [("oracle_kpm_moments", ": 2.0 * hv[i] - prev[i];", ": hv[i] - prev[i];")],
    "kpm_sign": [("oracle_kpm_moments", ": 2.0 * hv[i] - prev[i];", ": 2.0 * hv[i] + prev[i];")],
    "kpm_first_step_doubled": [("oracle_kpm_moments", "(m == 0) ? hv[i]", "(m == 0) ? 2.0 * hv[i]")],
    "kpm_dot_with_prev": [("oracle_kpm_moments", "d = d + V0[i * R + r] * cur[i];",
                           "d = d + V0[i * R + r] * prev[i];")],
    "lanczos_no_prev": [("oracle_lanczos", "w[i] = w[i] - b_prev * prev[i];", "w[i] = w[i];")],
    "lanczos_alpha_sign": [("oracle_lanczos", "w[i] = w[i] - a * cur[i];", "w[i] = w[i] + a * cur[i];")],
    "lanczos_beta_not_sqrt": [("oracle_lanczos", "b = sqrt(b);", "b = b;")],
    "lanczos_unnormalised_start": [("oracle_lanczos", "cur[i] = nq > 0.0 ? q[i] / nq : 0.0;",
                                    "cur[i] = q[i];")],
    "bf16_ties_away": [("oracle_round_bf16", "nearbyint(q)", "round(q)")],
    "bf16_precision": [("oracle_round_bf16", "E - 7;", "E - 8;")],
    "bf16_subnormal_threshold": [("oracle_round_bf16", "(E < -126)", "(E < -127)")],
    "bf16_decode_bias": [("oracle_bf16_to_f64", "e - 127", "e - 126")],
    "f32_truncate": [("oracle_round_f32", "out[i] = (float)in[i];",
                      "{ float f = (float)in[i]; if (fabs((double)f) > fabs(in[i])) f = nextafterf(f, 0.0f); out[i] = f; }")],
}


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


def _build_and_run(src: str, outdir, name: str):
    c = os.path.join(outdir, name + ".c")
    so = os.path.join(outdir, name + ".so")
    with open(c, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", so, c, "-lm"])
    pins_py = os.path.join(os.path.dirname(pins.__file__), "pins.py")
    return subprocess.run([sys.executable, pins_py, so], capture_output=True, text=True, timeout=300)


def test_unaltered_copy_passes(mutant_dir):
    src = open(ORACLE_SRC).read()
    r = _build_and_run(src, str(mutant_dir), "unaltered")
    assert r.returncode == 0 and "ALL-PASS" in r.stdout, r.stdout + r.stderr


@pytest.mark.parametrize("name", sorted(MUTANTS) + ["transposed"])
def test_mutant_rejected(name, mutant_dir):
    src = open(ORACLE_SRC).read()
    if name == "transposed":
        a, b = _function_span(src, "oracle_spmv")
        src = src[:a] + TRANSPOSED + src[b:]
    else:
        src = _mutate(src, MUTANTS[name])
    r = _build_and_run(src, str(mutant_dir), name)
    assert r.returncode != 0 and "ALL-PASS" not in r.stdout, (name, r.stdout)
