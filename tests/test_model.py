"""The benchmark's performance model against the numbers the paper prints
(tests/golden/paper_model.txt, each with its passage)."""
import math

import pytest

import bench
import pins

G = {k: (float(v[0]), float(v[1])) for k, v in pins.read_golden("paper_model.txt").items()}


def approx(name, value):
    target, tol = G[name]
    assert abs(value - target) <= tol + 1e-12, (name, value, target, tol)


def test_eq1_balance_and_limits():
    approx("balance_nnzr15_kappa0", bench.code_balance(15))
    approx("perf_limit_spmv_bw_gflops", bench.perf_limit(G["spmv_bw_GBs"][0], 15))
    approx("perf_limit_stream_gflops", bench.perf_limit(G["stream_bw_GBs"][0], 15))
    approx("spmv_fraction_of_stream", G["spmv_bw_GBs"][0] / G["stream_bw_GBs"][0])


def test_kappa_hmep():
    k = bench.kappa_from(G["spmv_bw_GBs"][0], G["measured_gflops"][0], 15)
    approx("kappa_hmep", k)
    approx("extra_bytes_per_row_hmep", k * 15)
    approx("rhs_loads_hmep", bench.rhs_loads(k, 15))
    k2 = G["kappa_hmep_electronic"][0]
    approx("extra_transfer_increase", k2 / k - 1)
    approx("perf_drop_hmep_electronic", bench.code_balance(15, k2) / bench.code_balance(15, k) - 1)


def test_kappa_uhbr():
    nnzr = G["uhbr_nnzr"][0]
    k = bench.kappa_from(G["uhbr_bw_GBs"][0], G["uhbr_gflops"][0], nnzr)
    approx("kappa_uhbr", k)
    approx("rhs_loads_uhbr", bench.rhs_loads(G["kappa_uhbr"][0], nnzr))


def test_eq2_split_penalty():
    approx("split_penalty_nnzr7", bench.code_balance_split(7) / bench.code_balance(7) - 1)
    approx("split_penalty_nnzr15", bench.code_balance_split(15) / bench.code_balance(15) - 1)
    # with kappa > 0 the penalty is smaller
    assert bench.code_balance_split(7, 2.0) / bench.code_balance(7, 2.0) < \
        bench.code_balance_split(7) / bench.code_balance(7)


def test_node_ratio_and_matrix_dimension():
    approx("node_ratio_hmep_electronic", 3.89 / 4.34)
    # six electrons on six sites (3 up, 3 down) times 15 phonons on six sites
    approx("hh_dimension", math.comb(6, 3) ** 2 * math.comb(15 + 6 - 1, 6 - 1))


def test_gpu_byte_model():
    # Eq. (1) counts 12 + 24/N_nzr bytes per entry; the GPU model adds row_ptr
    n, nnz = 4_096_000, 109_215_352
    b = bench.algorithmic_bytes(n, n, nnz, "f64")
    assert b == 1_425_272_228
    assert b == 12 * nnz + 28 * n + 4  # 12 + (4 + 24)/N_nzr bytes per entry, plus one row_ptr end
    assert bench.algorithmic_bytes(n, n, nnz, "f32") == 939_258_820
    assert bench.algorithmic_bytes(n, n, nnz, "bf16") == 720_828_116
    assert bench.algorithmic_bytes(n, n, nnz, "f32f64") == 988_410_820
    # k right-hand sides: matrix once, vectors k times
    assert bench.algorithmic_bytes(10, 10, 30, "f64", 4) == 30 * 12 + 44 + 10 * 4 * 8 + 2 * 10 * 4 * 8
    assert bench.split_extra_bytes(1000) == 1000 * 24 + 4
