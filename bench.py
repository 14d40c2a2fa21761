#!/usr/bin/env python3
"""Benchmark of the CRS spMV path on one MI355X.

Headline (the JSON line's `value`): C = C + A*B in FP64 on the 3D 27-point
stencil on a 160^3 grid (N = 4,096,000 rows, 109,215,352 stored entries,
entries 26 / -1 perturbed by U[-0.01, 0.01], B ~ U[-1, 1]), inputs resident
in HBM.  One step is one spmv_run over the whole matrix.  The same run also
measures the other paths of the library (reduced precision, the irregular
matrix and its local / nonlocal split with the halo copy overlapped, block
right-hand sides, the 512-matrix batch) and reports them under "paths".

Performance model (Sect. 1.2 and Sect. 3.4 of Schubert, Fehske, Hager,
Wellein 2011): code balance Eq. (1) B = 6 + 12/N_nzr + kappa/2 bytes/flop,
split balance Eq. (2) 6 + 20/N_nzr + kappa/2; kappa from measured bandwidth
and performance as in Sect. 2.  On the GPU the algorithmic byte count also
includes row_ptr (4 bytes per row) and C is read and written once (no
write-allocate): nnz*(s_val + 4) + 4*(N+1) + n_cols*k*s_x + 2*N*k*s_c.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only headline]
       python bench.py --only headline --plan '{...}'   (headline with a fixed plan)
       python bench.py --pmc-pass --plan '{...}'         (headline kernel + copy
                                          calibration, for rocprofv3 --pmc runs)
       python bench.py --summarize-pmc FETCH_DIR WRITE_DIR OUT PLAN
       python bench.py --summarize-stats STATS_CSV OUT COMMAND
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1106_5908_amd", "csrc", "kernels.hip")

VAL_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f32f64": 4}
VEC_BYTES = {"f64": 8, "f32": 4, "bf16": 4, "f32f64": 8}


# ----------------------------------------------------------------------------
# Performance model
# ----------------------------------------------------------------------------

def code_balance(nnzr: float, kappa: float = 0.0) -> float:
    """Eq. (1): bytes per flop of the CRS kernel, FP64 val, 4-byte indices."""
    return 6.0 + 12.0 / nnzr + kappa / 2.0


def code_balance_split(nnzr: float, kappa: float = 0.0) -> float:
    """Eq. (2): the split kernel writes the result vector twice."""
    return 6.0 + 20.0 / nnzr + kappa / 2.0


def perf_limit(bw_gbs: float, nnzr: float, kappa: float = 0.0) -> float:
    """Upper performance limit in GFlop/s: bandwidth over code balance."""
    return bw_gbs / code_balance(nnzr, kappa)


def kappa_from(bw_gbs: float, perf_gflops: float, nnzr: float) -> float:
    """kappa from the measured bandwidth and performance (Sect. 2)."""
    return 2.0 * (bw_gbs / perf_gflops - 6.0 - 12.0 / nnzr)


def rhs_loads(kappa: float, nnzr: float) -> float:
    """How many times B is loaded: once plus kappa*N_nzr/8 extra loads."""
    return 1.0 + kappa * nnzr / 8.0


def algorithmic_bytes(n_rows: int, n_cols: int, nnz: int, prec: str = "f64", k: int = 1) -> int:
    """Bytes one call must move at kappa = 0 (val, col_idx, row_ptr, B once,
    C read and written once)."""
    sv, sx = VAL_BYTES[prec], VEC_BYTES[prec]
    return nnz * (sv + 4) + 4 * (n_rows + 1) + n_cols * k * sx + 2 * n_rows * k * sx


def split_extra_bytes(n_nl_rows: int, prec: str = "f64") -> int:
    """Extra bytes of the split: the nonlocal rows' C read and written again,
    their row id and their row_ptr entry."""
    sc = VEC_BYTES[prec]
    return n_nl_rows * (2 * sc + 8) + 4


def kappa_gpu(bytes_measured: float, flops: float, model_bytes: float) -> float:
    """GPU analogue of kappa: twice the measured bytes per flop above the
    kappa = 0 model."""
    return 2.0 * (bytes_measured / flops - model_bytes / flops)


# ----------------------------------------------------------------------------
# Timing helpers
# ----------------------------------------------------------------------------

def time_launches(fn, steps: int, warmup: int):
    """Run fn() warmup times, then `steps` times between one event pair
    (ms_per_step: nothing else is enqueued between the calls), then `steps`
    more times with an event pair around each call for the per-call spread
    (mean, p10, p50, p90).  Events on torch's current stream, the stream the
    library launches on.  Returns dict of ms figures."""
    import torch

    s = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(s)
    for _ in range(steps):
        fn()
    t1.record(s)
    torch.cuda.synchronize()
    total = t0.elapsed_time(t1)
    # per-call events cost the runtime a little time of their own, so they
    # stay out of the series above
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(s)
    for i in range(steps):
        fn()
        ev[i + 1].record(s)
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return {
        "ms_per_step": total / steps,
        "mean_ms": float(per.mean()),
        "p10_ms": float(np.percentile(per, 10)),
        "p50_ms": float(np.percentile(per, 50)),
        "p90_ms": float(np.percentile(per, 90)),
    }


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(plan, workload: str = "27pt160"):
    """HBM bytes per product from the committed counter summary of `workload`
    taken with the current kernel source and this plan (a plan dict, or for
    the split {"local": ..., "nonlocal": ...}); None if there is none."""
    for path in sorted(glob.glob(os.path.join(PROFILES, "traffic_*.txt"))):
        try:
            with open(path) as f:
                t = json.load(f)
        except (OSError, ValueError):
            continue
        if (t.get("kernel_sha") == kernel_hash() and _same_traffic_plan(t.get("plan"), plan)
                and t.get("pmc_workload", "27pt160") == workload):
            return t.get("traffic_bytes")
    return None


def _same_traffic_plan(a, b):
    """Plans that launch the same kernels: equal, or, for the split under the
    merged-tail schedule (which runs no nonlocal kernel), the same local plan."""
    from paper_1106_5908_amd import spmv

    merged = spmv.SPMV_SCHEDULE_OVERLAP_MERGED
    if isinstance(a, dict) and isinstance(b, dict) and a.get("schedule") == b.get("schedule") == merged:
        return a.get("local") == b.get("local")
    return a == b


def traffic_report(traffic, model_bytes: float, flops: float):
    """Measured bytes, their ratio to the algorithmic bytes and the GPU kappa
    (Eq. (1) analogue); all None without a matching counter summary."""
    if not traffic:
        return {"traffic_bytes": None, "traffic_over_model": None, "kappa_gpu": None}
    return {"traffic_bytes": traffic, "traffic_over_model": traffic / model_bytes,
            "kappa_gpu": kappa_gpu(traffic, flops, model_bytes)}


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


SETUP_TIMES = {}


def make_handle(A, prec="f64", tune=True):
    """Handle with the plan the autotuner picks (the cache is bypassed, so
    every run tunes); the ingest and tuning times of the last call are kept
    in SETUP_TIMES."""
    from paper_1106_5908_amd import spmv

    t0 = time.perf_counter()
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec=prec,
                             flags=spmv.SPMV_FLAG_NO_TUNE_CACHE)
    t1 = time.perf_counter()
    if tune:
        spmv.spmv_tune(h, 1)
    SETUP_TIMES.update(create_ms=(t1 - t0) * 1e3, tune_ms=(time.perf_counter() - t1) * 1e3 if tune else 0.0)
    return h


def dev_vec(a, prec):
    import torch

    dt = torch.float64 if VEC_BYTES[prec] == 8 else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dt)


def normalized_err(A, x, got, ref=None, den=None):
    import oracle

    if ref is None:
        ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x)
    e = oracle.normalized_error(got, ref, den)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.abs(got - ref) / np.abs(ref)
        # condition number of entry i of the sum: (|c0| + sum |a||b|) / |c_i|
        cond = den / np.abs(ref)
    fin = np.isfinite(rel)
    above = fin & (rel > 1e-12)
    out = {
        "max_normalized_err": float(e.max()),
        "max_rel_err": float(rel[fin].max()) if fin.any() else 0.0,
        "n_rel_err_above_1e-12": int(above.sum()),
    }
    if above.any():
        # A8: where the plain relative error exceeds 1e-12 the entry's sum is
        # ill-conditioned; rel <= cond * normalised error for each of them
        c = cond[above]
        out["cond_of_rel_err_above_1e-12"] = {
            "min": float(c.min()), "median": float(np.median(c)), "max": float(c.max()),
            "max_rel_over_cond_times_norm_err": float(np.max(rel[above] / (c * np.maximum(e[above], 1e-300)))),
            "worst_entries": [{"row": int(i), "rel_err": float(rel[i]), "cond": float(cond[i]),
                               "normalized_err": float(e[i])}
                              for i in np.flatnonzero(above)[np.argsort(-rel[above])[:5]]],
        }
    return out, ref, den


def bound(prec: str, n: int) -> float:
    u64, u32, u16 = 2.0 ** -53, 2.0 ** -24, 2.0 ** -8
    return {"f64": 1e-12, "f32": (n + 3) * u32, "bf16": u16 + (n + 3) * u32,
            "f32f64": u32 + (n + 2) * u64}[prec]


def run_spmv_path(A, x, prec, steps, warmup, label, ref=None, den=None, tune=True, plan=None):
    """Time spmv_run on one matrix in one precision; check the first result.
    With `plan` given the autotuner is skipped and that plan is used."""
    import torch

    from paper_1106_5908_amd import spmv

    h = make_handle(A, prec, tune and plan is None)
    setup = dict(SETUP_TIMES)
    if plan is not None:
        spmv.spmv_set_plan(h, **plan)
    B = dev_vec(x, prec)
    C = torch.zeros(A.n_rows, dtype=B.dtype, device="cuda")
    spmv.spmv_run(h, B, C)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    # the first call's output is checked against the oracle after the timed
    # calls, so the device does not idle between them while the CPU works
    t = time_launches(lambda: spmv.spmv_run(h, B, C), steps, warmup)
    err, ref, den = normalized_err(A, x, got, ref, den)
    plan = spmv.spmv_get_plan(h)
    spmv.spmv_destroy(h)
    del B, C
    torch.cuda.empty_cache()
    mb = algorithmic_bytes(A.n_rows, A.n_cols, A.nnz, prec)
    flops = 2.0 * A.nnz
    n = int(np.diff(A.row_ptr).max())
    out = {
        "path": label, "prec": prec, "gflops": flops / (t["ms_per_step"] * 1e6),
        "model_GBs": mb / (t["ms_per_step"] * 1e6), "model_bytes": mb, **t, **err,
        "err_bound": bound(prec, n), "within_bound": err["max_normalized_err"] <= bound(prec, n),
        "plan": plan, "ingest_ms": setup["create_ms"], "tune_ms": setup["tune_ms"],
    }
    log(f"{label} {prec}: {out['gflops']:.0f} GFlop/s, {out['model_GBs']:.0f} GB/s model, "
        f"err {err['max_normalized_err']:.2e}")
    return out, ref, den


def measure_bandwidth(steps=20):
    """Copy and triad probes over 3 x 2^27 doubles (the STREAM role)."""
    import torch

    from paper_1106_5908_amd import spmv

    n = 1 << 27
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.rand(n, dtype=torch.float64, device="cuda")
    sums = torch.empty(spmv.read_sums_needed(n), dtype=torch.float64, device="cuda")
    tc = time_launches(lambda: spmv.spmv_probe_copy(a, b), steps, 3)
    tt = time_launches(lambda: spmv.spmv_probe_triad(a, b, c, 3.0), steps, 3)
    tr = time_launches(lambda: spmv.spmv_probe_read(b, sums), steps, 3)
    out = {"copy_GBs": 2 * 8 * n / (tc["p50_ms"] * 1e6), "triad_GBs": 3 * 8 * n / (tt["p50_ms"] * 1e6),
           "read_GBs": 8 * n / (tr["p50_ms"] * 1e6), "copy_bytes": 2 * 8 * n, "copy_ms": tc["p50_ms"],
           "array_doubles": n}
    del a, b, c, sums
    torch.cuda.empty_cache()
    log(f"bandwidth probes: copy {out['copy_GBs']:.0f} GB/s, triad {out['triad_GBs']:.0f} GB/s, "
        f"read {out['read_GBs']:.0f} GB/s")
    return out


def kpm_path(A, R: int = 8, M: int = 64, reps: int = 5):
    """Chebyshev moments of the kernel polynomial method (Sect. 1.3's
    polynomial-expansion methods) on the matrix scaled into [-1, 1] by its
    largest absolute row sum: R start vectors, M moments, ceil(M/2) block
    products per call, timed against one block product alone."""
    import torch

    from paper_1106_5908_amd import spmv
    from workloads import gen

    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    g = float(np.bincount(rows, weights=np.abs(A.val), minlength=A.n_rows).max())
    val = A.val / (1.01 * g)
    del rows
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, val, A.n_cols,
                             flags=spmv.SPMV_FLAG_NO_TUNE_CACHE)
    del val
    spmv.spmv_tune(h, R)
    V0 = torch.from_numpy(gen.uniform_vector(A.n_rows * R, gen.rng_for(30, R)).reshape(A.n_rows, R)).to("cuda")
    W1, W2 = torch.empty_like(V0), torch.empty_like(V0)
    mu = spmv.spmv_kpm_moments(h, V0, M, W1, W2)
    torch.cuda.synchronize()
    norm2 = (V0 * V0).sum(dim=0)
    bounded = bool(torch.all(mu.abs() <= norm2[None, :] * (1 + 1e-9)).item())
    t = time_launches(lambda: spmv.spmv_kpm_moments(h, V0, M, W1, W2), reps, 1)
    tb = time_launches(lambda: spmv.spmv_run_block(h, V0, W1), reps, 1)
    products = (M + 1) // 2
    flops = 2.0 * A.nnz * R * products
    out = {"R": R, "M": M, "products_per_call": products, "ms_per_call": t["p50_ms"],
           "moments_per_s": M * R / (t["p50_ms"] * 1e-3), "gflops_products": flops / (t["p50_ms"] * 1e6),
           "block_product_ms": tb["p50_ms"], "frac_time_in_products": products * tb["p50_ms"] / t["p50_ms"],
           "moments_bounded_by_norm": bounded, "scale": 1.01 * g,
           "plan_block": spmv.spmv_get_block_plan(h, R)}
    spmv.spmv_destroy(h)
    del V0, W1, W2, mu
    torch.cuda.empty_cache()
    log(f"kpm: {M} moments x {R} vectors in {t['p50_ms']:.2f} ms ({products} block products of "
        f"{tb['p50_ms']:.2f} ms; {out['frac_time_in_products'] * 100:.0f}% of the time), "
        f"{out['gflops_products']:.0f} GFlop/s")
    return out


def lanczos_path(A, spmv_ms: float, m: int = 100, reps: int = 3):
    """Lanczos (the eigensolver Sect. 1.3 names first) on the symmetric
    irregular matrix: m steps enqueued at once, timed per call; the per-step
    cost against one product; the extreme Ritz values of the m x m
    tridiagonal matrix."""
    import torch
    from scipy.linalg import eigvalsh_tridiagonal

    from paper_1106_5908_amd import spmv
    from workloads import gen

    h = make_handle(A, "f64")
    q = torch.from_numpy(gen.uniform_vector(A.n_rows, gen.rng_for(43, 0))).to("cuda")
    V1, V2 = torch.empty_like(q), torch.empty_like(q)
    a, b = spmv.spmv_lanczos(h, q, m, V1, V2)
    torch.cuda.synchronize()
    t = time_launches(lambda: spmv.spmv_lanczos(h, q, m, V1, V2), reps, 1)
    a2, b2 = spmv.spmv_lanczos(h, q, m, V1, V2)
    torch.cuda.synchronize()
    same = bool(torch.equal(a, a2) and torch.equal(b, b2))
    an, bn = a.cpu().numpy(), b.cpu().numpy()
    ritz = eigvalsh_tridiagonal(an, bn[:-1])
    spmv.spmv_destroy(h)
    del q, V1, V2
    torch.cuda.empty_cache()
    step = t["p50_ms"] / m
    out = {"m": m, "ms_per_call": t["p50_ms"], "ms_per_step": step, "spmv_ms": spmv_ms,
           "frac_time_in_products": spmv_ms / step, "ritz_min": float(ritz[0]), "ritz_max": float(ritz[-1]),
           "last_beta": float(bn[-1]), "repeatable": same,
           "gflops_products": 2.0 * A.nnz * m / (t["p50_ms"] * 1e6)}
    log(f"lanczos: {m} steps in {t['p50_ms']:.1f} ms ({step * 1e3:.0f} us per step against "
        f"{spmv_ms * 1e3:.0f} us per product), Ritz range [{ritz[0]:.4f}, {ritz[-1]:.4f}]")
    return out


def atomic_probe(nnz27: int, n27: int, head_ms: float, iters: int = 100):
    """FP64 atomic-add throughput into a 32 MB vector, coalesced and
    scattered, and what it implies for the transposed half of a symmetric
    (upper-triangle) product of the 27-point matrix: (nnz - N) / 2
    contributions scattered into C."""
    import torch

    from paper_1106_5908_amd import spmv

    C = torch.zeros(1 << 22, dtype=torch.float64, device="cuda")
    out = {"target_bytes": 8 << 22}
    for name, sc in (("coalesced", False), ("scattered", True)):
        C.zero_()
        made = spmv.spmv_probe_atomic(C, sc, iters)
        torch.cuda.synchronize()
        exact = float(C.sum().item()) == float(made)
        t = time_launches(lambda: spmv.spmv_probe_atomic(C, sc, iters), 5, 2)
        out[name] = {"atomics": made, "ms": t["p50_ms"], "G_per_s": made / (t["p50_ms"] * 1e6),
                     "sum_exact": exact}
    contrib = (nnz27 - n27) // 2
    out["sym27_transposed_contributions"] = contrib
    out["sym27_scatter_ms_at_coalesced_rate"] = contrib / (out["coalesced"]["G_per_s"] * 1e6)
    out["sym27_scatter_ms_at_scattered_rate"] = contrib / (out["scattered"]["G_per_s"] * 1e6)
    out["full_storage_product_ms"] = head_ms
    del C
    torch.cuda.empty_cache()
    log(f"atomics: coalesced {out['coalesced']['G_per_s']:.1f} G/s, scattered "
        f"{out['scattered']['G_per_s']:.1f} G/s; symmetric 27-point scatter alone >= "
        f"{out['sym27_scatter_ms_at_coalesced_rate'] * 1e3:.0f} us vs full product "
        f"{head_ms * 1e3:.0f} us")
    return out


def symmetric_path(steps: int, warmup: int):
    """Symmetric storage (Sect. 1.3.1) on the unperturbed 27-point 160^3
    stencil (26 / -1, exactly symmetric): the upper triangle with the
    transposed half scattered by atomic adds, against full storage of the
    same matrix, each with its tuned plan.  Integer B, so both results are
    exact and must agree bit for bit."""
    import torch

    from paper_1106_5908_amd import spmv
    from workloads import gen

    A = gen.stencil_27pt_3d(160)
    U = gen.upper_triangle(A)
    x = gen.integer_vector(A.n_cols, gen.rng_for(2, 11), vmax=8)
    B = torch.from_numpy(x).to("cuda")
    hf = make_handle(A)
    hs = spmv.spmv_create_sym_crs(U.row_ptr, U.col_idx, U.val, flags=spmv.SPMV_FLAG_NO_TUNE_CACHE)
    spmv.spmv_tune(hs)
    out = {"n_rows": A.n_rows, "nnz_full": A.nnz, "nnz_upper": U.nnz,
           "plan_full": spmv.spmv_get_plan(hf), "plan_symmetric": spmv.spmv_get_plan(hs)}
    res = []
    for h in (hf, hs):
        C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
        spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        res.append(C.cpu().numpy())
        t = time_launches(lambda: spmv.spmv_run(h, B, C), steps, warmup)
        out["full_ms" if h is hf else "symmetric_ms"] = t["p50_ms"]
    out["results_bit_exact"] = bool(np.array_equal(res[0], res[1]))
    out["matrix_bytes_full"] = A.nnz * 12 + 4 * (A.n_rows + 1)
    out["matrix_bytes_symmetric"] = U.nnz * 12 + 4 * (A.n_rows + 1)
    out["symmetric_over_full_time"] = out["symmetric_ms"] / out["full_ms"]
    spmv.spmv_destroy(hs)
    spmv.spmv_destroy(hf)
    del A, U, B
    torch.cuda.empty_cache()
    log(f"symmetric storage: {out['symmetric_ms'] * 1e3:.0f} us against {out['full_ms'] * 1e3:.0f} us "
        f"for full storage ({out['nnz_upper']} of {out['nnz_full']} entries stored; results equal: "
        f"{out['results_bit_exact']})")
    return out


def split_paths(A, x, steps, warmup):
    """The three schedules of Fig. 5 on one GPU: (a) blocking halo copy then
    the unsplit kernel, (b) split kernels with the copy serialised on the
    compute stream, (c) split kernels with the copy overlapped; then the full
    exchange cycle with the send side, overlapped (d) and serialised (e)."""
    import torch

    import oracle
    from paper_1106_5908_amd import spmv
    from workloads import gen

    hb = gen.halo_begin(A.n_cols)
    n_halo = A.n_cols - hb
    halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory()
    B = dev_vec(x, "f64")
    C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    a = make_handle(A, "f64")
    s = spmv.spmv_split_local_nonlocal(a, hb)
    spmv.spmv_tune(s, 1)
    info = spmv.spmv_get_info(s)
    res = {"halo_begin": hb, "n_halo": n_halo, "halo_bytes": 8 * n_halo,
           "nnz_local": info["nnz_local"], "nnz_nonlocal": info["nnz_nonlocal"],
           "n_nonlocal_rows": info["n_nonlocal_rows"]}
    # parity of the overlapped split (first call), against the unsplit oracle
    Bc = B.clone()
    Bc[hb:] = float("nan")
    spmv.spmv_run(s, Bc, C, halo)
    torch.cuda.synchronize()
    ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
    den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x)
    res["split_max_normalized_err"] = float(oracle.normalized_error(C.cpu().numpy(), ref, den).max())

    def mode_a():
        B[hb:].copy_(halo, non_blocking=False)
        spmv.spmv_run(a, B, C)

    def mode_b():
        spmv.spmv_run(s, B, C, halo)

    # the schedule spmv_tune chose, then each schedule set explicitly
    tct = time_launches(mode_b, steps, warmup)
    tkt = time_launches(lambda: spmv.spmv_run(s, B, C), steps, warmup)
    spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_SERIAL)
    tb = time_launches(mode_b, steps, warmup)
    spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_OVERLAP_MERGED)
    tc2 = time_launches(mode_b, steps, warmup)
    tk2 = time_launches(lambda: spmv.spmv_run(s, B, C), steps, warmup)  # merged tail, resident
    spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL)
    tc1 = time_launches(mode_b, steps, warmup)
    tk1 = time_launches(lambda: spmv.spmv_run(s, B, C), steps, warmup)  # nonlocal beside local, resident
    spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_OVERLAP)
    tc = time_launches(mode_b, steps, warmup)
    ta = time_launches(mode_a, steps, warmup)
    tk = time_launches(lambda: spmv.spmv_run(s, B, C), steps, warmup)  # halo resident
    tu = time_launches(lambda: spmv.spmv_run(a, B, C), steps, warmup)  # unsplit kernel only
    flops = 2.0 * A.nnz
    mb = algorithmic_bytes(A.n_rows, A.n_cols, A.nnz, "f64")
    res.update({
        "a_blocking_copy_then_unsplit_ms": ta["p50_ms"],
        "b_split_serial_copy_ms": tb["p50_ms"],
        "c_split_overlap_copy_ms": tc["p50_ms"],
        "c_nonlocal_beside_local_ms": tc1["p50_ms"],
        "c_merged_tail_ms": tc2["p50_ms"],
        "c_tuned_schedule_ms": tct["p50_ms"],
        "split_kernels_only_ms": tk["p50_ms"],
        "split_kernels_nonlocal_beside_local_ms": tk1["p50_ms"],
        "split_kernels_merged_tail_ms": tk2["p50_ms"],
        "split_kernels_tuned_schedule_ms": tkt["p50_ms"],
        "unsplit_kernel_only_ms": tu["p50_ms"],
        "c_gflops": flops / (tc["p50_ms"] * 1e6),
        "split_model_bytes": mb + split_extra_bytes(info["n_nonlocal_rows"]),
        "split_model_penalty": split_extra_bytes(info["n_nonlocal_rows"]) / mb,
        # the split as the library runs it (the schedule spmv_tune chose),
        # then each schedule on its own
        "split_kernel_penalty": tkt["p50_ms"] / tu["p50_ms"] - 1.0,
        "split_kernel_penalty_ordered": tk["p50_ms"] / tu["p50_ms"] - 1.0,
        "split_kernel_penalty_nonlocal_beside_local": tk1["p50_ms"] / tu["p50_ms"] - 1.0,
        "split_kernel_penalty_merged_tail": tk2["p50_ms"] / tu["p50_ms"] - 1.0,
        "c_tuned_gflops": flops / (tct["p50_ms"] * 1e6),
        "overlap_speedup_vs_a": ta["p50_ms"] / tc["p50_ms"],
        "overlap_speedup_vs_b": tb["p50_ms"] / tc["p50_ms"],
        "plans": {"local": spmv.spmv_get_plan(s, spmv.SPMV_PART_MAIN),
                  "nonlocal": spmv.spmv_get_plan(s, spmv.SPMV_PART_NONLOCAL)},
    })
    res.update(traffic_report(read_traffic(res["plans"], "irregular8M-split"),
                              res["split_model_bytes"], flops))
    merged = traffic_report(read_traffic({**res["plans"], "schedule": spmv.SPMV_SCHEDULE_OVERLAP_MERGED},
                                         "irregular8M-split"), mb, flops)
    res.update({f"{k}_merged_tail": v for k, v in merged.items()})
    log(f"split: (a) {ta['p50_ms']*1e3:.0f} us, (b) {tb['p50_ms']*1e3:.0f} us, "
        f"(c) {tc['p50_ms']*1e3:.0f} us (nonlocal beside local {tc1['p50_ms']*1e3:.0f} us, merged tail "
        f"{tc2['p50_ms']*1e3:.0f} us, tuned {tct['p50_ms']*1e3:.0f} us), kernels only "
        f"{tk['p50_ms']*1e3:.0f} us (nonlocal beside local {tk1['p50_ms']*1e3:.0f} us, merged tail "
        f"{tk2['p50_ms']*1e3:.0f} us, tuned {tkt['p50_ms']*1e3:.0f} us), unsplit {tu['p50_ms']*1e3:.0f} us")

    # (d) / (e): the whole exchange cycle of task mode (Sect. 3.5): the send
    # list of the symmetric matrix is packed and copied to pinned host memory
    # beside the halo copy and the local part (d), or all in order (e)
    n_send = spmv.spmv_send_list_symmetric(s)
    send = torch.empty(n_send, dtype=torch.float64).pin_memory()
    idx = spmv.spmv_export(s, spmv.SPMV_ARR_SEND_IDX)
    spmv.spmv_run_exchange(s, B, C, halo, send)
    torch.cuda.synchronize()
    exact = bool(np.array_equal(send.numpy().view(np.uint64),
                                oracle.pack(idx, x).view(np.uint64)))
    td = time_launches(lambda: spmv.spmv_run_exchange(s, B, C, halo, send), steps, warmup)
    spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_SERIAL)
    te = time_launches(lambda: spmv.spmv_run_exchange(s, B, C, halo, send), steps, warmup)
    spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_OVERLAP)
    res.update({
        "n_send": n_send, "send_bytes": 8 * n_send, "send_buffer_bit_exact": exact,
        "d_exchange_overlap_ms": td["p50_ms"], "e_exchange_serial_ms": te["p50_ms"],
        "exchange_cost_over_c": td["p50_ms"] / tc["p50_ms"] - 1.0,
        "exchange_overlap_speedup_vs_e": te["p50_ms"] / td["p50_ms"],
    })
    log(f"exchange: (d) {td['p50_ms']*1e3:.0f} us overlapped, (e) {te['p50_ms']*1e3:.0f} us "
        f"serial, {n_send} elements sent, bit-exact {exact}")

    # per-phase events (copy, local, nonlocal, send) of schedules (c) and (d)
    def phases(call, reps=20):
        spmv.spmv_set_phase_timing(s, True)
        rows = []
        for _ in range(reps):
            call()
            torch.cuda.synchronize()
            rows.append(spmv.spmv_phase_times(s))
        spmv.spmv_set_phase_timing(s, False)
        out = {}
        for ph in spmv.PHASES:
            spans = [r[ph] for r in rows if r[ph]]
            if spans:
                out[ph + "_ms"] = float(np.median([b - a for a, b in spans]))
        for ph in ("copy", "send"):
            ov = []
            for r in rows:
                if r[ph] and r["local"]:
                    (a0, a1), (l0, l1) = r[ph], r["local"]
                    ov.append(max(0.0, min(a1, l1) - max(a0, l0)) / max(a1 - a0, 1e-9))
            if ov:
                out[ph + "_share_during_local"] = float(np.median(ov))
        out["call_ms"] = float(np.median([max(v[1] for v in r.values() if v) for r in rows]))
        return out

    res["phases_c"] = phases(lambda: spmv.spmv_run(s, B, C, halo))
    res["phases_d"] = phases(lambda: spmv.spmv_run_exchange(s, B, C, halo, send))
    pc, pd = res["phases_c"], res["phases_d"]
    log(f"phases (c): copy {pc['copy_ms']*1e3:.0f} us ({pc['copy_share_during_local']*100:.0f}% under the "
        f"local part {pc['local_ms']*1e3:.0f} us), nonlocal {pc['nonlocal_ms']*1e3:.0f} us; (d): send "
        f"{pd['send_ms']*1e3:.0f} us ({pd['send_share_during_local']*100:.0f}% under the local part)")
    spmv.spmv_destroy(s)
    spmv.spmv_destroy(a)
    del B, C, Bc
    torch.cuda.empty_cache()
    return res, ref, den


def block_paths(A, steps, warmup, fp64_ms):
    import torch

    import oracle
    from paper_1106_5908_amd import spmv
    from workloads import gen

    out = []
    rows = np.random.default_rng(5).integers(0, A.n_rows, size=2000)
    for prec in ("f64", "f32"):
        h = make_handle(A, prec, tune=False)
        for k in gen.BLOCK_KS:
            spmv.spmv_tune(h, k)
            X = gen.block_rhs(A.n_cols, k)
            dt = torch.float64 if prec == "f64" else torch.float32
            B = torch.from_numpy(X).to("cuda", dtype=dt)
            C = torch.zeros((A.n_rows, k), dtype=dt, device="cuda")
            spmv.spmv_run_block(h, B, C)
            torch.cuda.synchronize()
            got = C[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
            errs = []
            for t in range(k):
                xt = np.ascontiguousarray(X[:, t])
                ref = oracle.spmv_rows(rows, A.row_ptr, A.col_idx, A.val, xt)
                den = oracle.spmv_rows(rows, A.row_ptr, A.col_idx, np.abs(A.val), np.abs(xt))
                errs.append(float(oracle.normalized_error(got[:, t], ref, den).max()))
            tm = time_launches(lambda: spmv.spmv_run_block(h, B, C), steps, warmup)
            flops = 2.0 * A.nnz * k
            mb = algorithmic_bytes(A.n_rows, A.n_cols, A.nnz, prec, k)
            n = int(np.diff(A.row_ptr).max())
            r = {"path": f"block k={k}", "prec": prec, "k": k,
                 "gflops": flops / (tm["ms_per_step"] * 1e6),
                 "model_GBs": mb / (tm["ms_per_step"] * 1e6), "model_bytes": mb, **tm,
                 "max_normalized_err_sampled": max(errs), "err_bound": bound(prec, n),
                 "speedup_vs_k_fp64_calls": k * fp64_ms / tm["ms_per_step"],
                 "plan": spmv.spmv_get_block_plan(h, k)}
            if prec == "f64":
                r.update(traffic_report(read_traffic(r["plan"], f"irregular8M-k{k}"), mb, flops))
            log(f"block k={k} {prec}: {r['gflops']:.0f} GFlop/s, x{r['speedup_vs_k_fp64_calls']:.2f} "
                f"vs k FP64 calls, err {max(errs):.1e}")
            out.append(r)
            del B, C
            torch.cuda.empty_cache()
        spmv.spmv_destroy(h)
    return out


def _sorted_block_rows(n_rows: int, n_cu: int, rmax: int = 16384) -> int:
    """Rows per block of the library's sorted-block layout (FP64 sums): rmax,
    or for a part of at least three quarters of a round (rmax rows on every
    CU) the size that makes whole rounds of one block per CU."""
    full = rmax * n_cu
    if 4 * n_rows < 3 * full:
        return rmax
    rounds = -(-n_rows // full)
    return min(rmax, -(-n_rows // (rounds * n_cu)))


def _plan_index_stream(A, plan, fused_rows: int = 512, n_cu: int = 256):
    """The order in which a plan's launches gather B, as (col_idx order,
    launch cuts): the matrix order without panels; with K diagonal panels
    (the library's slices of col - row) panel after panel, one launch each;
    for the fused-panel kernel row block after row block (fused_rows rows),
    each block's panels in turn, in one launch; for the sorted-block kernel
    block after block (the library's FP64 block size), each block's entries
    by column from the first multiple of the widest block span above the
    block's lowest column, wrapping round (the library further deals them
    into chunks with distinct rows, which moves a few entries by a chunk)."""
    K = int(plan.get("panels", 1))
    n = A.nnz
    if plan.get("kernel") == 6:
        if n == 0:
            return A.col_idx, [0, 0]
        R = _sorted_block_rows(A.n_rows, n_cu)
        bounds = A.row_ptr[np.arange(0, A.n_rows, R)].astype(np.int64)  # first entry per block
        counts = np.diff(np.append(bounds, n))
        keep = counts > 0
        col = A.col_idx.astype(np.int64)
        lo = np.minimum.reduceat(col, bounds[keep])
        hi = np.maximum.reduceat(col, bounds[keep])
        period = int((hi - lo + 1).max())
        s0 = -(-lo // period) * period
        start = np.where((s0 > lo) & (s0 <= hi), s0, lo)
        blk = np.repeat(np.arange(keep.sum(), dtype=np.int64), counts[keep])
        st = start[blk]
        # per block: columns at or above the start first, then the wrapped ones
        key = (blk << 42) + np.where(col >= st, col - st, col - st + (1 << 41))
        return A.col_idx[np.argsort(key, kind="stable")], [0, n]
    if K <= 1:
        return A.col_idx, [0, n]
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    d = A.col_idx.astype(np.int64) - rows
    dmin, dmax = int(d.min()), int(d.max())
    p = np.clip(((d - dmin) * K) // (dmax - dmin + 1), 0, K - 1)
    if plan.get("kernel") == 5:
        key = (rows // fused_rows) * K + p
        return A.col_idx[np.argsort(key, kind="stable")], [0, n]
    cuts = [0] + [int(c) for c in np.cumsum(np.bincount(p, minlength=K))]
    return A.col_idx[np.argsort(p, kind="stable")], cuts


def gather_ceiling(A, plan, kernel_ms, block_rows, reps: int = 10):
    """What the irregular matrix's gathers of B cost on their own
    (spmv_probe_gather): random 8-byte gathers, as many as the matrix has
    entries, from a 1 MiB window (resident in every XCD's L2) and from a
    1 GiB one (HBM); then the index stream of the tuned plan itself (the
    matrix's col_idx in the plan's launch order and XCD placement) against
    the product's own time; and the same for each block product, gathering
    its k doubles per index.  `block_rows`: [(k, plan, ms)]."""
    import torch

    from paper_1106_5908_amd import spmv

    n = A.nnz
    rng = np.random.default_rng(1106)

    def timed(fn):
        return time_launches(fn, reps, 3)["p50_ms"]

    out = {"gathers": n}
    src = torch.rand(1 << 27, dtype=torch.float64, device="cuda")
    for name, rows in (("l2_1MiB", 1 << 17), ("hbm_1GiB", 1 << 27)):
        idx = torch.from_numpy(rng.integers(0, rows, size=n).astype(np.int32)).cuda()
        t = timed(lambda: spmv.spmv_probe_gather(src[:rows], idx, 1, True))
        out[f"random_{name}_ms"] = t
        out[f"random_{name}_G_per_s"] = n / (t * 1e6)
        del idx
    del src

    n_cu = torch.cuda.get_device_properties(0).multi_processor_count

    def own(width, pl):
        order, cuts = _plan_index_stream(A, pl, n_cu=n_cu)
        idx = torch.from_numpy(np.ascontiguousarray(order)).cuda()
        Bw = torch.rand(A.n_cols * width, dtype=torch.float64, device="cuda")
        rm = bool(pl.get("xcd_remap", 1))

        def run():
            for a, b in zip(cuts[:-1], cuts[1:]):
                spmv.spmv_probe_gather(Bw, idx[a:b], width, rm)

        t = timed(run)
        del idx, Bw
        torch.cuda.empty_cache()
        return t

    t_own = own(1, plan)
    out.update({"plan": plan, "own_stream_ms": t_own, "kernel_ms": kernel_ms,
                "kernel_rate_over_own_stream": t_own / kernel_ms,
                "kernel_rate_over_l2_random": out["random_l2_1MiB_ms"] / kernel_ms})
    blocks = []
    for k, pl, ms in block_rows:
        t = own(k, pl)
        blocks.append({"k": k, "plan": pl, "own_stream_ms": t, "kernel_ms": ms,
                       "kernel_rate_over_own_stream": t / ms})
    out["blocks_f64"] = blocks
    log(f"gather ceiling: L2-resident random {out['random_l2_1MiB_ms'] * 1e3:.0f} us, HBM random "
        f"{out['random_hbm_1GiB_ms'] * 1e3:.0f} us, own stream {t_own * 1e3:.0f} us vs kernel "
        f"{kernel_ms * 1e3:.0f} us ({out['kernel_rate_over_own_stream'] * 100:.0f}%); blocks " +
        ", ".join(f"k={b['k']} {b['own_stream_ms'] * 1e3:.0f}/{b['kernel_ms'] * 1e3:.0f} us" for b in blocks))
    return out


def batch_paths(steps, warmup):
    import torch

    import oracle
    from paper_1106_5908_amd import spmv
    from workloads import gen

    t0 = time.time()
    mem = gen.workload_c5_batch()
    log(f"batch generated in {time.time() - t0:.1f}s")
    n_rows = sum(A.n_rows for A, _ in mem)
    n_cols = sum(A.n_cols for A, _ in mem)
    nnz = sum(A.nnz for A, _ in mem)
    xs = np.concatenate([x for _, x in mem])
    h = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols) for A, _ in mem],
                               flags=spmv.SPMV_FLAG_NO_TUNE_CACHE)
    spmv.spmv_tune(h, 1)
    B = dev_vec(xs, "f64")
    C = torch.zeros(n_rows, dtype=torch.float64, device="cuda")
    spmv.spmv_run(h, B, C)
    torch.cuda.synchronize()
    got = C.cpu().numpy()
    worst = 0.0
    off_r = off_c = 0
    for A, x in mem[:64]:
        ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x)
        worst = max(worst, float(oracle.normalized_error(got[off_r:off_r + A.n_rows], ref, den).max()))
        off_r += A.n_rows
        off_c += A.n_cols
    res = {"members": len(mem), "n_rows": n_rows, "nnz": nnz,
           "max_normalized_err_first64": worst, "plan": spmv.spmv_get_plan(h)}
    flops = 2.0 * nnz
    mb = algorithmic_bytes(n_rows, n_cols, nnz, "f64") + 4 * len(mem)
    tuned = spmv.spmv_get_plan(h)
    for kname, kern in (("queue", spmv.SPMV_KERNEL_STREAM), ("tilegrid", spmv.SPMV_KERNEL_TILE_GRID)):
        spmv.spmv_set_plan(h, kernel=kern)
        for name, sch in (("graph", spmv.SPMV_SCHEDULE_BATCH_GRAPH), ("direct", spmv.SPMV_SCHEDULE_BATCH_DIRECT)):
            spmv.spmv_set_schedule(h, sch)
            tm = time_launches(lambda: spmv.spmv_run(h, B, C), steps, warmup)
            res[f"{kname}_{name}_ms"] = tm["p50_ms"]
            res[f"{kname}_{name}_gflops"] = flops / (tm["ms_per_step"] * 1e6)
    spmv.spmv_set_plan(h, **tuned)
    spmv.spmv_set_schedule(h, spmv.SPMV_SCHEDULE_BATCH_GRAPH)
    tm = time_launches(lambda: spmv.spmv_run(h, B, C), steps, warmup)
    res["graph_ms"] = tm["p50_ms"]
    res["graph_gflops"] = flops / (tm["ms_per_step"] * 1e6)
    res["graph_model_GBs"] = mb / (tm["ms_per_step"] * 1e6)
    spmv.spmv_destroy(h)
    # baseline: one plain launch per member
    hs = [make_handle(A, "f64", tune=False) for A, _ in mem]
    views = []
    off_r = off_c = 0
    for A, _ in mem:
        views.append((B[off_c:off_c + A.n_cols], C[off_r:off_r + A.n_rows]))
        off_r += A.n_rows
        off_c += A.n_cols

    def per_member():
        for hh, (b, c) in zip(hs, views):
            spmv.spmv_run(hh, b, c)

    tm = time_launches(per_member, max(3, steps // 5), 2)
    res["per_member_launches_ms"] = tm["p50_ms"]
    res["per_member_gflops"] = flops / (tm["ms_per_step"] * 1e6)
    res["graph_speedup_vs_per_member"] = tm["p50_ms"] / res["graph_ms"]
    res["model_bytes"] = mb
    for hh in hs:
        spmv.spmv_destroy(hh)
    log(f"batch: tuned graph {res['graph_ms']*1e3:.0f} us ({res['graph_gflops']:.0f} GFlop/s, "
        f"kernel {res['plan']['kernel']}); queue graph {res['queue_graph_ms']*1e3:.0f} us, "
        f"queue direct {res['queue_direct_ms']*1e3:.0f} us, tile-grid graph {res['tilegrid_graph_ms']*1e3:.0f} us, "
        f"tile-grid direct {res['tilegrid_direct_ms']*1e3:.0f} us, per-member launches "
        f"{res['per_member_launches_ms']*1e3:.0f} us")
    del B, C, views
    torch.cuda.empty_cache()
    return res


def overlap_probe(reps: int = 5):
    """Asynchrony test, the one-GPU analogue of Listing 2 / Fig. 4: a spin
    kernel of length T on the compute stream while an 80 MB host-to-device
    copy runs on a second stream, from pinned and from pageable memory.  A
    truly asynchronous copy gives total ~ max(T, T_copy); a serialised one
    T + T_copy."""
    import torch

    from paper_1106_5908_amd import spmv

    n = 10_000_000  # 80 MB of doubles, the message size of Listing 2
    dst = torch.empty(n, dtype=torch.float64, device="cuda")
    pinned = torch.rand(n, dtype=torch.float64).pin_memory()
    pageable = torch.rand(n, dtype=torch.float64)
    s0 = torch.cuda.current_stream()
    s1 = torch.cuda.Stream()

    def total(spin_ms, src):
        best = 1e30
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if spin_ms > 0:
                spmv.spmv_probe_spin(int(spin_ms * 1e6), s0)
            if src is not None:
                with torch.cuda.stream(s1):
                    dst.copy_(src, non_blocking=True)
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) * 1e3)
        return best

    t_copy = total(0, pinned)
    t_copy_pageable = total(0, pageable)
    rows = []
    for f in (0.5, 1.0, 2.0):
        T = f * t_copy
        rows.append({"spin_ms": T, "spin_alone_ms": total(T, None), "pinned_total_ms": total(T, pinned),
                     "pageable_total_ms": total(T, pageable)})
    out = {"copy_bytes": 8 * n, "pinned_copy_ms": t_copy, "pageable_copy_ms": t_copy_pageable,
           "pinned_GBs": 8 * n / (t_copy * 1e6), "rows": rows}
    log(f"overlap probe: 80 MB copy {t_copy:.2f} ms pinned, {t_copy_pageable:.2f} ms pageable; " +
        "; ".join(f"T={r['spin_ms']:.2f}: pinned {r['pinned_total_ms']:.2f}, pageable "
                  f"{r['pageable_total_ms']:.2f} ms" for r in rows))
    del dst, pinned, pageable
    return out


def cpu_baseline(A, x, budget_s: float = 12.0):
    """The oracle (sequential, one core) on repeated full passes of the
    headline matrix until about budget_s seconds of CPU work."""
    import oracle

    oracle.spmv(A.row_ptr[:2], A.col_idx[:A.row_ptr[1]], A.val[:A.row_ptr[1]], x)  # load
    # one thread, pinned to one host core for the duration of the timing
    before = os.sched_getaffinity(0)
    core = min(before)
    os.sched_setaffinity(0, {core})
    try:
        reps = 0
        t0 = time.perf_counter()
        while True:
            oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget_s or reps >= 400:
                break
    finally:
        os.sched_setaffinity(0, before)
    gflops = 2.0 * A.nnz * reps / el / 1e9
    log(f"cpu oracle: {reps} passes in {el:.1f}s on core {core} -> {gflops:.3f} GFlop/s")
    return {"value": gflops, "unit": "GFlop/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full sequential passes of the 27-point 160^3 FP64 product "
                      f"({el:.1f} s, one thread pinned to host core {core})"}


def cold_headline(A, x, plan, reps: int = 20):
    """The headline product with caches flushed before every call: a 1 GiB
    buffer (four times the 256 MB MALL) is overwritten between calls,
    outside the timed interval; each call is timed alone with an event pair."""
    import torch

    from paper_1106_5908_amd import spmv

    h = make_handle(A, "f64", tune=False)
    spmv.spmv_set_plan(h, **plan)
    B = dev_vec(x, "f64")
    C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    scrub = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    times = []
    for i in range(reps + 2):
        scrub.fill_(float(i))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        spmv.spmv_run(h, B, C)
        e1.record(s)
        torch.cuda.synchronize()
        if i >= 2:
            times.append(e0.elapsed_time(e1))
    spmv.spmv_destroy(h)
    del B, C, scrub
    torch.cuda.empty_cache()
    t = np.array(times)
    med = float(np.median(t))
    mb = algorithmic_bytes(A.n_rows, A.n_cols, A.nnz, "f64")
    out = {"median_ms": med, "p10_ms": float(np.percentile(t, 10)),
           "p90_ms": float(np.percentile(t, 90)), "gflops": 2.0 * A.nnz / (med * 1e6),
           "model_GBs": mb / (med * 1e6), "scrub_bytes": 1 << 30, "calls": reps, "plan": plan}
    log(f"27pt160 cold: {out['gflops']:.0f} GFlop/s ({med * 1e3:.1f} us)")
    return out


OMP_SRC = os.path.join(ROOT, "bench_omp.c")
OMP_LIB = os.path.join(ROOT, "bench_omp.so")


def build_omp(force: bool = False) -> str:
    """Compile the OpenMP CPU baseline (bench_omp.c) with gcc."""
    if force or not os.path.exists(OMP_LIB) or os.path.getmtime(OMP_LIB) < os.path.getmtime(OMP_SRC):
        tmp = OMP_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-Wall", "-shared", "-fPIC", "-o", tmp,
                               OMP_SRC])
        os.replace(tmp, OMP_LIB)
    return OMP_LIB


def cpu_omp(A, x, ref, den, reps: int = 10, triad_n: int = 1 << 26):
    """The paper's node-level CRS (OpenMP rows, static schedule, first touch)
    and the triad on all host threads; kappa of the host from the two."""
    import ctypes

    import oracle

    lib = ctypes.CDLL(build_omp())
    lib.omp_crs_bench.restype = ctypes.c_double
    lib.omp_crs_bench.argtypes = [ctypes.c_int64, ctypes.c_int64] + [ctypes.c_void_p] * 4 + [
        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.omp_triad_bench.restype = ctypes.c_double
    lib.omp_triad_bench.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    xv = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(A.n_rows, dtype=np.float64)
    nt = ctypes.c_int(0)
    sec = lib.omp_crs_bench(A.n_rows, A.n_cols, rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                            xv.ctypes.data, reps, y.ctypes.data, ctypes.byref(nt))
    if sec <= 0:
        return None
    nt2 = ctypes.c_int(0)
    triad = lib.omp_triad_bench(triad_n, 10, ctypes.byref(nt2))
    perf = 2.0 * A.nnz / sec / 1e9
    nnzr = A.nnz / A.n_rows
    wa = triad * 4.0 / 3.0
    err = float(oracle.normalized_error(y, ref, den).max())
    out = {"gflops": perf, "median_ms": sec * 1e3, "threads": nt.value,
           "cores_visible": len(os.sched_getaffinity(0)),
           "model_GBs": algorithmic_bytes(A.n_rows, A.n_cols, A.nnz, "f64") / sec / 1e9,
           "triad_GBs": triad, "triad_GBs_with_write_allocate": wa,
           "kappa": kappa_from(wa, perf, nnzr), "max_normalized_err": err,
           "schedule": "OpenMP static over rows, first-touch placement"}
    log(f"cpu OpenMP CRS: {perf:.2f} GFlop/s on {nt.value} threads, triad {triad:.1f} GB/s")
    return out


# ----------------------------------------------------------------------------
# rocprofv3 counter passes
# ----------------------------------------------------------------------------

PMC_WORKLOADS = {
    # name: (matrix, k, description)
    "27pt160": ("c2", 1, "27-point 160^3 FP64"),
    "irregular8M": ("c3", 1, "irregular 8M FP64"),
    "irregular8M-split": ("c3", 0, "irregular 8M FP64, local and nonlocal parts (h = 7,520,000)"),
    "irregular8M-k4": ("c3", 4, "irregular 8M FP64, block of k = 4"),
    "irregular8M-k8": ("c3", 8, "irregular 8M FP64, block of k = 8"),
    "irregular8M-k16": ("c3", 16, "irregular 8M FP64, block of k = 16"),
}


def pmc_pass(steps: int, plan_json: str | None, workload: str = "27pt160"):
    """The product of one workload `steps` times with the given plan (no
    tuning, so the profile holds only these dispatches), then a copy of 2^27
    doubles (the calibration kernel of known size), each bracketed by
    synchronisation.  Block workloads take the block plan (block_kt set);
    the split takes {"local": plan, "nonlocal": plan} (and optionally
    "schedule": a split schedule) and runs with the halo resident (no
    copy)."""
    import torch

    from paper_1106_5908_amd import spmv
    from workloads import gen

    mat, k, _ = PMC_WORKLOADS[workload]
    A, x = gen.workload_c2() if mat == "c2" else gen.workload_c3()
    h = make_handle(A, "f64", tune=False)
    handles = [h]
    plan = json.loads(plan_json) if plan_json else None
    if k == 0:
        s = spmv.spmv_split_local_nonlocal(h, gen.halo_begin(A.n_cols))
        handles.append(s)
        if plan:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, **plan["local"])
            spmv.spmv_set_plan(s, spmv.SPMV_PART_NONLOCAL, **plan["nonlocal"])
            if "schedule" in plan:
                spmv.spmv_set_schedule(s, plan["schedule"])
        B = dev_vec(x, "f64")
        C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
        call = lambda: spmv.spmv_run(s, B, C)  # noqa: E731
        got = {"local": spmv.spmv_get_plan(s, spmv.SPMV_PART_MAIN),
               "nonlocal": spmv.spmv_get_plan(s, spmv.SPMV_PART_NONLOCAL)}
        if plan and "schedule" in plan:
            got["schedule"] = plan["schedule"]
    else:
        if plan:
            spmv.spmv_set_plan(h, **plan)
        if k == 1:
            B = dev_vec(x, "f64")
            C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
            call = lambda: spmv.spmv_run(h, B, C)  # noqa: E731
            got = spmv.spmv_get_plan(h)
        else:
            B = torch.from_numpy(gen.block_rhs(A.n_cols, k)).to("cuda")
            C = torch.zeros((A.n_rows, k), dtype=torch.float64, device="cuda")
            call = lambda: spmv.spmv_run_block(h, B, C)  # noqa: E731
            got = spmv.spmv_get_block_plan(h, k)
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    # release the handles (their device arrays) before the calibration copy
    # and before the process ends
    for hh in reversed(handles):
        spmv.spmv_destroy(hh)
    del B, C, call
    n = 1 << 27
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    for _ in range(3):
        spmv.spmv_probe_copy(a, b)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
    print(json.dumps({"pmc_pass": "done", "workload": workload, "plan": got,
                      "copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n}), flush=True)


def trace_pass(steps: int):
    """The split product of the irregular 8M matrix for a rocprofv3
    --kernel-trace --memory-copy-trace run: `steps` calls of schedule (c)
    (halo copy overlapped with the local part) and then `steps` calls of the
    exchange cycle (d), each call alone between synchronisations, each
    series preceded by a 2 ms spin kernel that marks it in the trace."""
    import time

    import torch

    from paper_1106_5908_amd import spmv
    from workloads import gen

    A, x = gen.workload_c3()
    hb = gen.halo_begin(A.n_cols)
    a = make_handle(A, "f64", tune=False)
    s = spmv.spmv_split_local_nonlocal(a, hb)
    spmv.spmv_tune(s, 1)
    n_send = spmv.spmv_send_list_symmetric(s)
    halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory()
    send = torch.empty(n_send, dtype=torch.float64).pin_memory()
    B = dev_vec(x, "f64")
    C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    try:
        for call in (lambda: spmv.spmv_run(s, B, C, halo),
                     lambda: spmv.spmv_run_exchange(s, B, C, halo, send)):
            call()
            torch.cuda.synchronize()
            spmv.spmv_probe_spin(2_000_000)
            torch.cuda.synchronize()
            for _ in range(steps):
                time.sleep(0.002)
                call()
                torch.cuda.synchronize()
        plans = {"local": spmv.spmv_get_plan(s, spmv.SPMV_PART_MAIN),
                 "nonlocal": spmv.spmv_get_plan(s, spmv.SPMV_PART_NONLOCAL)}
    finally:
        # Nothing of the library outlives this function: the split handle's
        # copy and send streams and events, both handles' device arrays and
        # the pinned host buffers are all released before the process ends.
        torch.cuda.synchronize()
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
        del halo, send, B, C
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    print(json.dumps({"trace_pass": "done", "steps": steps, "halo_bytes": 8 * (A.n_cols - hb),
                      "send_bytes": 8 * n_send, "plans": plans}), flush=True)


def phases_pass(steps: int, out_path: str, command: str):
    """Per-call phase events of the split product of the irregular 8M matrix
    (the library's own hipEvents on the GPU clock, spmv_phase_times): `steps`
    calls of schedule (c) (halo copy overlapped with the local part), of (c)
    with the nonlocal part beside the local part, of (c) with the last
    blocks run over local and nonlocal entries together (their interval is
    reported as the nonlocal one), and of the exchange cycle (d), each call
    alone; writes one line per call with
    the halo copy, local, nonlocal and send intervals (us from the call's
    start), the share of the copy (and of the send side) that ran while the
    local part ran, and whether the copy ended before the local part and the
    nonlocal part started after both."""
    import torch

    from paper_1106_5908_amd import spmv
    from workloads import gen

    A, x = gen.workload_c3()
    hb = gen.halo_begin(A.n_cols)
    a = make_handle(A, "f64", tune=False)
    s = spmv.spmv_split_local_nonlocal(a, hb)
    spmv.spmv_tune(s, 1)
    n_send = spmv.spmv_send_list_symmetric(s)
    halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory()
    send = torch.empty(n_send, dtype=torch.float64).pin_memory()
    B = dev_vec(x, "f64")
    C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    lines = ["# Split product of the irregular 8M matrix, one line per call: phase intervals from the "
             "library's events (spmv_set_phase_timing / spmv_phase_times), us from the call's start",
             f"# command: {command}",
             f"# plans: local {spmv.spmv_get_plan(s, spmv.SPMV_PART_MAIN)}, "
             f"nonlocal {spmv.spmv_get_plan(s, spmv.SPMV_PART_NONLOCAL)}; halo {8 * (A.n_cols - hb)} B, "
             f"send buffer {8 * n_send} B"]
    summary = {}
    try:
        spmv.spmv_set_phase_timing(s, True)
        for name, sched, call in (
                ("c_split_overlap", spmv.SPMV_SCHEDULE_OVERLAP, lambda: spmv.spmv_run(s, B, C, halo)),
                ("c_split_beside", spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL,
                 lambda: spmv.spmv_run(s, B, C, halo)),
                ("c_split_merged", spmv.SPMV_SCHEDULE_OVERLAP_MERGED,
                 lambda: spmv.spmv_run(s, B, C, halo)),
                ("d_exchange_overlap", spmv.SPMV_SCHEDULE_OVERLAP,
                 lambda: spmv.spmv_run_exchange(s, B, C, halo, send))):
            spmv.spmv_set_schedule(s, sched)
            sorted_local = spmv.spmv_get_plan(s, spmv.SPMV_PART_MAIN)["kernel"] == \
                spmv.SPMV_KERNEL_SORTED_BLOCKS
            beside = sched == spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL or \
                (sched == spmv.SPMV_SCHEDULE_OVERLAP_MERGED and sorted_local)
            for _ in range(3):
                call()
            torch.cuda.synchronize()
            lines.append(f"{name}:")
            def share(a, lo):
                return max(0.0, min(a[1], lo[1]) - max(a[0], lo[0])) / max(a[1] - a[0], 1e-9)

            ends_first = after = 0
            shares, send_shares = [], []
            for i in range(steps):
                call()
                torch.cuda.synchronize()
                t = spmv.spmv_phase_times(s)
                us = {k: (v[0] * 1e3, v[1] * 1e3) for k, v in t.items() if v}
                c, lo, nl = us["copy"], us["local"], us["nonlocal"]
                ok_end = c[1] <= lo[1]
                # beside: the nonlocal part within the local part's span, after the copy
                ok_after = (nl[0] >= c[1] and lo[0] <= nl[0] and nl[1] <= lo[1]) if beside else \
                    nl[0] >= max(c[1], lo[1])
                ends_first += ok_end
                after += ok_after
                shares.append(share(c, lo))
                snd = us.get("send")
                if snd:
                    send_shares.append(share(snd, lo))
                lines.append(f"  {i:3d}  copy [{c[0]:7.1f}, {c[1]:7.1f}]  local [{lo[0]:7.1f}, {lo[1]:7.1f}]  "
                             f"nonlocal [{nl[0]:7.1f}, {nl[1]:7.1f}]" +
                             (f"  send [{snd[0]:7.1f}, {snd[1]:7.1f}] {send_shares[-1] * 100:5.1f}%" if snd else "") +
                             f"  copy under local {shares[-1] * 100:5.1f}%")
            where = ("runs inside the local part's span, after the copy" if beside
                     else "starts after both")
            lines.append(f"  copy under the local part: median {np.median(shares) * 100:.1f}%, min "
                         f"{min(shares) * 100:.1f}%; the copy ends before the local part in {ends_first} of "
                         f"{steps} calls; the nonlocal part {where} in {after} of {steps}" +
                         (f"; send side under the local part: median {np.median(send_shares) * 100:.1f}%"
                          if send_shares else ""))
            summary[name] = {"calls": steps, "copy_share_under_local_median": float(np.median(shares)),
                             "copy_ends_before_local": ends_first,
                             ("nonlocal_inside_local" if beside else "nonlocal_after_both"): after}
        spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_OVERLAP)
        spmv.spmv_set_phase_timing(s, False)
    finally:
        torch.cuda.synchronize()
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
        del halo, send, B, C
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps({"phases_pass": "done", **summary}), flush=True)


def _template_args(name: str):
    i = name.find("<")
    if i < 0:
        return []
    depth, j = 0, i
    for j in range(i, len(name)):
        depth += name[j] == "<"
        depth -= name[j] == ">"
        if depth == 0:
            break
    return [t.strip() for t in name[i + 1:j].split(",")]


def summarize_trace(trace_dir, out_path, command):
    """Per call of the two series in a trace_pass trace: the halo copy
    (host to device), the send copy (device to host), the local-part kernels
    (everything launched before the first nonlocal-part kernel) and the
    nonlocal-part kernels (stream kernels with a row list), with how much of
    each copy ran while local kernels ran."""
    import csv

    def load(pattern):
        files = glob.glob(os.path.join(trace_dir, "**", pattern), recursive=True)
        if not files:
            raise SystemExit(f"no {pattern} under {trace_dir}")
        return list(csv.DictReader(open(files[0])))

    kern = load("*kernel_trace.csv")
    copies = load("*memory_copy_trace.csv")
    ev = []
    for r in kern:
        ev.append(("k", r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    dcol = next((c for c in copies[0].keys() if c.lower() in ("direction", "operation", "kind")), None)
    for r in copies:
        d = (r.get(dcol, "") if dcol else "").upper()
        kind = "h2d" if "HOST_TO_DEVICE" in d else ("d2h" if "DEVICE_TO_HOST" in d else "copy:" + d)
        ev.append((kind, d, int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    ev.sort(key=lambda e: e[2])
    marks = [i for i, e in enumerate(ev) if e[0] == "k" and "k_spin" in e[1]]
    if len(marks) < 2:
        raise SystemExit("trace lacks the two marker spins")
    series = {"c_split_overlap": ev[marks[0] + 1:marks[1]], "d_exchange": ev[marks[1] + 1:]}
    lines = ["# Halo copy against the local part: rocprofv3 kernel and memory-copy trace",
             f"# command: {command}",
             "# per call: copy durations, local-part span, the share of each copy that ran while "
             "local kernels ran, and the gap from the halo copy's end to the first nonlocal kernel"]
    result = {}
    per_call = {}
    for name, evs in series.items():
        calls, cur, last_end = [], [], None
        for e in evs:
            if last_end is not None and e[2] - last_end > 1_000_000:  # 1 ms gap between calls
                calls.append(cur)
                cur = []
            cur.append(e)
            last_end = max(last_end or 0, e[3])
        if cur:
            calls.append(cur)
        rows = []
        for c in calls:
            ks = [e for e in c if e[0] == "k"]
            nl = [e for e in ks if ("k_stream" in e[1] or "k_staged" in e[1])
                  and _template_args(e[1])[-1:] == ["true"]]
            first_nl = min((e[2] for e in nl), default=None)
            loc = [e for e in ks if first_nl is None or e[2] < first_nl]
            loc = [e for e in loc if "k_pack" not in e[1]]
            h2d = [e for e in c if e[0] == "h2d"]
            d2h = [e for e in c if e[0] == "d2h"]
            if not loc or not h2d:
                continue
            l0, l1 = min(e[2] for e in loc), max(e[3] for e in loc)

            def overlap(cp):
                tot = sum(e[3] - e[2] for e in cp)
                ov = sum(max(0, min(e[3], l1) - max(e[2], l0)) for e in cp)
                return tot, (ov / tot if tot else 0.0)

            th, oh = overlap(h2d)
            td, od = overlap(d2h) if d2h else (0, 0.0)
            gap = (first_nl - max(e[3] for e in h2d)) if first_nl is not None else None
            span = max(e[3] for e in c) - min(e[2] for e in c)
            rows.append((th, oh, td, od, l1 - l0, gap, span))
            t0c = min(e[2] for e in c)
            nl_end = max((e[3] for e in nl), default=None)
            per_call.setdefault(name, []).append(
                (min(e[2] for e in h2d) - t0c, max(e[3] for e in h2d) - t0c, l0 - t0c, l1 - t0c,
                 None if first_nl is None else first_nl - t0c,
                 None if nl_end is None else nl_end - t0c, oh))
        if not rows:
            continue
        a = np.array([[r[0], r[1], r[2], r[3], r[4], r[6]] for r in rows], dtype=float)
        gaps = [r[5] for r in rows if r[5] is not None]
        med = np.median(a, axis=0)
        result[name] = {"calls": len(rows), "h2d_us": med[0] / 1e3, "h2d_overlap": med[1],
                        "d2h_us": med[2] / 1e3, "d2h_overlap": med[3], "local_span_us": med[4] / 1e3,
                        "call_span_us": med[5] / 1e3,
                        "min_gap_copy_end_to_nonlocal_us": (min(gaps) / 1e3 if gaps else None)}
        lines.append(f"{name}: {len(rows)} calls (medians)")
        lines.append(f"  halo copy H2D {med[0] / 1e3:8.1f} us, {med[1] * 100:5.1f}% of it during local kernels")
        if med[2]:
            lines.append(f"  send copy D2H {med[2] / 1e3:8.1f} us, {med[3] * 100:5.1f}% of it during local kernels")
        lines.append(f"  local part {med[4] / 1e3:8.1f} us, whole call {med[5] / 1e3:8.1f} us")
        if gaps:
            lines.append(f"  first nonlocal kernel starts {min(gaps) / 1e3:.1f} us (min) after the halo copy ends")
        lines.append("  per call, us from the call's first event: halo copy [start, end], local kernels "
                     "[start, end], nonlocal kernels [start, end], share of the copy under the local kernels")
        for i, (c0, c1, l0_, l1_, n0, n1, o) in enumerate(per_call.get(name, [])):
            nl_txt = "-" if n0 is None else f"[{n0 / 1e3:7.1f}, {n1 / 1e3:7.1f}]"
            lines.append(f"  {i:3d}  copy [{c0 / 1e3:7.1f}, {c1 / 1e3:7.1f}]  local [{l0_ / 1e3:7.1f}, "
                         f"{l1_ / 1e3:7.1f}]  nonlocal {nl_txt}  {o * 100:5.1f}%")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    print(json.dumps(result))


def _counter_rows(d):
    import csv

    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def summarize_pmc(fetch_dir, write_dir, out_path, plan_json, workload="27pt160", steps="10"):
    """FETCH_SIZE / WRITE_SIZE (KiB) of the product, summed over its kernel
    dispatches (several with diagonal panels) and divided by the number of
    products, scaled by the same counters' reading for the copy kernel of
    known size."""
    steps = int(steps)

    def per_kernel(rows, counter):
        acc = {}
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"]
            spmv_kernel = "spmv::" in name and any(
                k in name for k in ("k_stream", "k_staged", "k_vector", "k_block", "k_fused", "k_sorted"))
            key = "spmv" if spmv_kernel else ("copy" if "k_copy" in name else None)
            if key is None:
                continue
            acc.setdefault((key, r["Dispatch_Id"]), 0.0)
            acc[(key, r["Dispatch_Id"])] += float(r["Counter_Value"])
        out = {}
        for (key, _), v in acc.items():
            out.setdefault(key, []).append(v)
        return {"copy": float(np.median(out["copy"])), "spmv": float(np.sum(out["spmv"])) / steps,
                "spmv_dispatches": len(out["spmv"])}

    fetch = per_kernel(_counter_rows(fetch_dir), "FETCH_SIZE")
    write = per_kernel(_counter_rows(write_dir), "WRITE_SIZE")
    copy_bytes = 8 * (1 << 27)
    f_fac = copy_bytes / (fetch["copy"] * 1024.0)
    w_fac = copy_bytes / (write["copy"] * 1024.0)
    fetch_b = fetch["spmv"] * 1024.0 * f_fac
    write_b = write["spmv"] * 1024.0 * w_fac
    mat, k, desc = PMC_WORKLOADS[workload]
    extra = 0
    if mat == "c2":
        n, nnz = 4096000, 109215352
    else:
        from workloads import gen

        import oracle

        A, _ = gen.workload_c3()
        n, nnz = A.n_rows, A.nnz
        from paper_1106_5908_amd import spmv

        # the merged-tail schedule reads every row's entries once, as the
        # unsplit product does: no row list and no second pass over C
        if k == 0 and json.loads(plan_json).get("schedule") != spmv.SPMV_SCHEDULE_OVERLAP_MERGED:
            parts = oracle.split(A.row_ptr, A.col_idx, A.val, gen.halo_begin(A.n_cols))
            extra = split_extra_bytes(int(parts["nl_rows"].size))
    wl = "" if workload == "27pt160" else f" --pmc-workload {workload}"
    res = {
        "kernel_sha": kernel_hash(), "plan": json.loads(plan_json),
        "workload": desc, "pmc_workload": workload,
        "fetch_kib_per_product": fetch["spmv"], "write_kib_per_product": write["spmv"],
        "dispatches_per_product": fetch["spmv_dispatches"] / steps,
        "copy_fetch_kib": fetch["copy"], "copy_write_kib": write["copy"],
        "fetch_scale": f_fac, "write_scale": w_fac,
        "traffic_bytes": fetch_b + write_b,
        "algorithmic_bytes": algorithmic_bytes(n, n, nnz, "f64", max(k, 1)) + extra,
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE -d <fetch_dir> -o p --output-format csv -- "
            f"python3 bench.py --pmc-pass --steps {steps} --plan '<plan>'{wl}",
            "rocprofv3 --pmc WRITE_SIZE -d <write_dir> -o p --output-format csv -- "
            f"python3 bench.py --pmc-pass --steps {steps} --plan '<plan>'{wl}",
            f"python3 bench.py --summarize-pmc <fetch_dir> <write_dir> <this file> '<plan>' {workload} {steps}",
        ],
        "scale_note": "counter KiB per dispatch x 1024 x (known bytes of the 2^27-double copy "
                      "/ the same counter's reading for that copy)",
    }
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def summarize_counters(out_path, command, *dirs):
    """Per-dispatch medians of every counter in one or more rocprofv3 --pmc
    runs of --pmc-pass, for the product's kernels and for the copy kernel,
    with the derived per-CU figures: busy cycles of the L1 address unit
    (TA_TA_BUSY_sum / 256 CUs) against the kernel's cycles
    (GRBM_GUI_ACTIVE / 8 XCDs), and L1 accesses per dispatch."""
    acc = {}
    for run, d in enumerate(dirs):  # dispatch numbers restart in every run
        for r in _counter_rows(d):
            name = r["Kernel_Name"]
            spmv_kernel = "spmv::" in name and any(
                k in name for k in ("k_stream", "k_staged", "k_vector", "k_block", "k_fused", "k_sorted"))
            key = "spmv" if spmv_kernel else ("copy" if "k_copy" in name else None)
            if key is None:
                continue
            d_acc = acc.setdefault((key, r["Counter_Name"]), {})
            d_acc[(run, r["Dispatch_Id"])] = d_acc.get((run, r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
    med = {}
    for (key, c), v in acc.items():
        med.setdefault(key, {})[c] = float(np.median(list(v.values())))
    lines = ["# rocprofv3 counters per dispatch (medians): the spMV kernel against the copy kernel",
             f"# command: {command}",
             f"# {'counter':40s} {'spmv':>16s} {'copy':>16s}"]
    for c in sorted(set(med.get("spmv", {})) | set(med.get("copy", {}))):
        lines.append(f"  {c:40s} {med.get('spmv', {}).get(c, float('nan')):16.1f} "
                     f"{med.get('copy', {}).get(c, float('nan')):16.1f}")
    for key in ("spmv", "copy"):
        m = med.get(key, {})
        if "TA_TA_BUSY_sum" in m and "GRBM_GUI_ACTIVE" in m:
            cyc = m["GRBM_GUI_ACTIVE"] / 8.0
            lines.append(f"# {key}: L1 address unit busy {m['TA_TA_BUSY_sum'] / 256.0 / cyc * 100:.0f}% of "
                         f"{cyc:.0f} cycles per CU")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_stats(stats_csv, out_path, command, kernel_filter=""):
    """Short text summary of a rocprofv3 --stats kernel table."""
    import csv

    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}",
             f"# {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_%':>8}  kernel"]
    for r in rows:
        name = r["Name"]
        if kernel_filter and kernel_filter not in name and "spmv" not in name:
            continue
        if len(name) > 110:
            name = name[:107] + "..."
        lines.append(f"  {int(r['Calls']):6d} {float(r['AverageNs'])/1e3:10.1f} {float(r['MinNs'])/1e3:10.1f} "
                     f"{float(r['MaxNs'])/1e3:10.1f} {float(r['Percentage']):8.2f}  {name}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# ----------------------------------------------------------------------------
# main
# ----------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--only", choices=["all", "headline"], default="all")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--pmc-pass", action="store_true")
    ap.add_argument("--plan", default=None,
                    help="plan (JSON) for the headline product instead of the autotuner's")
    ap.add_argument("--summarize-pmc", nargs="+",
                    metavar="FETCH_DIR WRITE_DIR OUT PLAN_JSON [WORKLOAD STEPS]")
    ap.add_argument("--pmc-workload", default="27pt160", choices=sorted(PMC_WORKLOADS))
    ap.add_argument("--summarize-stats", nargs=3, metavar=("STATS_CSV", "OUT", "COMMAND"))
    ap.add_argument("--trace-pass", action="store_true")
    ap.add_argument("--phases-pass", nargs=2, metavar=("OUT", "COMMAND"))
    ap.add_argument("--summarize-counters", nargs="+", metavar="OUT COMMAND DIR")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE_DIR", "OUT", "COMMAND"))
    args = ap.parse_args()

    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return 0
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats)
        return 0
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return 0
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X and has no "
              "multi-GPU mode (run with --gpus 1)", file=sys.stderr)
        return 2

    import torch

    from paper_1106_5908_amd import spmv
    from workloads import gen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    spmv.load()
    if args.pmc_pass:
        pmc_pass(args.steps, args.plan, args.pmc_workload)
        return 0
    if args.trace_pass:
        trace_pass(args.steps)
        return 0
    if args.phases_pass:
        phases_pass(args.steps, *args.phases_pass)
        return 0

    t_start = time.time()
    bw = measure_bandwidth()
    t0 = time.time()
    A2, x2 = gen.workload_c2()
    log(f"27-point 160^3 generated in {time.time() - t0:.1f}s ({A2.nnz} entries)")
    head, ref2, den2 = run_spmv_path(A2, x2, "f64", args.steps, args.warmup, "27pt160",
                                     plan=json.loads(args.plan) if args.plan else None)
    flops = 2.0 * A2.nnz
    mb = head["model_bytes"]
    traffic = read_traffic(head["plan"], "27pt160")
    # the same time basis as `value`: the timed region's events over K steps
    achieved = mb / (head["ms_per_step"] * 1e6)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    paths = {"bandwidth_probes": bw,
             "headline_detail": {**head, "frac_of_copy_bw": achieved / bw["copy_GBs"],
                                 "frac_of_triad_bw": achieved / bw["triad_GBs"],
                                 "frac_of_read_bw": achieved / bw["read_GBs"],
                                 "model_balance_B_per_flop": mb / flops,
                                 "paper_eq1_balance": code_balance(A2.nnz / A2.n_rows)}}
    if traffic:
        paths["headline_detail"]["kappa_gpu"] = kappa_gpu(traffic, flops, mb)

    if args.only == "all":
        paths["headline_cold"] = cold_headline(A2, x2, head["plan"])
        paths["atomic_probe"] = atomic_probe(A2.nnz, A2.n_rows, head["ms_per_step"])
        paths["symmetric_27pt160"] = symmetric_path(max(10, args.steps // 4), 3)
        prec_rows = []
        for prec in ("f32", "bf16", "f32f64"):
            r, _, _ = run_spmv_path(A2, x2, prec, args.steps, args.warmup, "27pt160", ref2, den2)
            r["speedup_vs_f64"] = head["ms_per_step"] / r["ms_per_step"]
            prec_rows.append(r)
        paths["precision_27pt160"] = prec_rows
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(A2, x2)
        paths["cpu_omp_27pt160"] = cpu_omp(A2, x2, ref2, den2)
    del A2, x2, ref2, den2

    if args.only == "all":
        t0 = time.time()
        A3, x3 = gen.workload_c3()
        log(f"irregular N=8e6 generated in {time.time() - t0:.1f}s ({A3.nnz} entries)")
        r3, ref3, den3 = run_spmv_path(A3, x3, "f64", args.steps, args.warmup, "irregular8M")
        r3.update(traffic_report(read_traffic(r3["plan"], "irregular8M"), r3["model_bytes"],
                                 2.0 * A3.nnz))
        paths["irregular8M_f64"] = r3
        # the stream kernel's best plan on this matrix (4 diagonal panels), the
        # reference the sorted-block kernel replaced and a second baseline for
        # the block products
        rs, _, _ = run_spmv_path(A3, x3, "f64", args.steps, args.warmup, "irregular8M stream",
                                 ref3, den3, plan=dict(kernel=1, tile_items=8, panels=4))
        r3["stream_panels4_ms_per_step"] = rs["ms_per_step"]
        r3["stream_panels4_gflops"] = rs["gflops"]
        r3["speedup_vs_stream_panels4"] = rs["ms_per_step"] / r3["ms_per_step"]
        p3 = []
        for prec in ("f32", "bf16", "f32f64"):
            r, _, _ = run_spmv_path(A3, x3, prec, args.steps, args.warmup, "irregular8M", ref3, den3)
            r["speedup_vs_f64"] = r3["ms_per_step"] / r["ms_per_step"]
            p3.append(r)
        paths["precision_irregular8M"] = p3
        del ref3, den3
        sp, _, _ = split_paths(A3, x3, max(20, args.steps // 2), args.warmup)
        paths["split_irregular8M"] = sp
        paths["overlap_probe"] = overlap_probe()
        paths["block_irregular8M"] = block_paths(A3, max(10, args.steps // 4), 3, r3["ms_per_step"])
        for b in paths["block_irregular8M"]:
            b["speedup_vs_k_fp64_stream_calls"] = b["k"] * rs["ms_per_step"] / b["ms_per_step"]
        paths["gather_ceiling_irregular8M"] = gather_ceiling(
            A3, r3["plan"], r3["ms_per_step"],
            [(b["k"], b["plan"], b["ms_per_step"]) for b in paths["block_irregular8M"] if b["prec"] == "f64"])
        paths["kpm_irregular8M"] = kpm_path(A3)
        paths["lanczos_irregular8M"] = lanczos_path(A3, r3["ms_per_step"])
        del A3, x3
        paths["batch_512_stencils"] = batch_paths(max(10, args.steps // 4), 3)

    # the paper's node-level figures, quoted with their hardware (context, not targets)
    paths["paper_context"] = {
        "hardware_socket": "Intel Xeon X5550 (Nehalem EP), one socket, 2.66 GHz, 3x DDR3-1333",
        "HMeP_socket": {"spmv_GBs": 18.1, "stream_triad_GBs": 21.2, "gflops": 2.25, "kappa": 2.5,
                        "model_limit_gflops": 2.66, "source": "Sect. 2"},
        "HMEp_socket": {"kappa": 3.79, "source": "Sect. 2"},
        "UHBR_socket": {"spmv_GBs": 18.9, "gflops": 2.99, "kappa": 0.43, "source": "Sect. 2"},
        "hardware_node": "2x Intel Xeon X5650 (Westmere EP)",
        "node_gflops": {"HMeP": 4.34, "HMEp": 3.89, "source": "Sect. 3.5"},
        "note": "another machine's figures, quoted as context; not targets",
    }
    line = {
        "metric": "spMV GFlop/s + achieved HBM GB/s vs 8 TB/s peak; FP64 vs mixed-prec at stated error",
        "value": flops / (head["ms_per_step"] * 1e6),
        "unit": "GFlop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D 27-point stencil 160^3, FP64 CRS, int32 indices, "
                               "C = C + A*B, inputs resident in HBM",
                   "n_rows": 4096000, "nnz": 109215352, "achieved_model_GBs": achieved,
                   "max_normalized_err": head["max_normalized_err"], "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "paths": paths,
        "wall_s": time.time() - t_start,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
