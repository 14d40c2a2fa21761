"""Send side of the exchange (pack kernel, device-to-host copy of the send
buffer, halo copy, split product) against the oracle, through the C
interface: send lists and send buffers bit for bit, C to the FP64 bound."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import FP64_TOL, assert_close, oracle_ref, to_dev
from paper_1106_5908_amd import spmv
from workloads import gen

pytestmark = pytest.mark.gpu

NOTUNE = spmv.SPMV_FLAG_NO_TUNE_CACHE
MODES = [spmv.SPMV_SCHEDULE_OVERLAP, spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL,
         spmv.SPMV_SCHEDULE_OVERLAP_MERGED, spmv.SPMV_SCHEDULE_SERIAL]


def _irregular():
    return gen.workload_c3(N=100_000)


def _handles(A, hb, prec="f64", flags=NOTUNE):
    a = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec=prec, flags=flags)
    return a, spmv.spmv_split_local_nonlocal(a, hb)


def _exchange(s, x, hb, prec, n_send, c0=None, pinned=True):
    """One spmv_run_exchange with a pinned halo and send buffer (C0 = c0, or
    zeros); returns (C, send buffer, receive area of B) on the host."""
    import torch

    xd = np.asarray(x, dtype=np.float64)
    Bh = xd.copy()
    Bh[hb:] = np.nan  # receive area: must be overwritten by the halo copy
    B = to_dev(Bh, prec)
    C = to_dev(np.zeros(s.n_rows) if c0 is None else c0, prec)
    halo = torch.from_numpy(np.ascontiguousarray(xd[hb:])).to(B.dtype)
    send = torch.full((n_send,), float("nan"), dtype=B.dtype)
    if pinned:
        halo, send = halo.pin_memory(), send.pin_memory()
    spmv.spmv_run_exchange(s, B, C, halo, send)
    torch.cuda.synchronize()
    return C.cpu().numpy().astype(np.float64), send.numpy().copy(), B[hb:].cpu().numpy()


@pytest.mark.parametrize("local_plan", [None, dict(kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS, tile_items=2)],
                         ids=["default", "sorted"])
@pytest.mark.parametrize("schedule", MODES)
def test_symmetric_send_list_and_cycle(schedule, local_plan):
    A, x = _irregular()
    hb = gen.halo_begin(A.n_cols)
    a, s = _handles(A, hb)
    try:
        if local_plan:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, **local_plan)
        n = spmv.spmv_send_list_symmetric(s)
        want = oracle.send_list_symmetric(A.row_ptr, A.col_idx, hb)
        assert n == want.size > 0
        assert np.array_equal(spmv.spmv_export(s, spmv.SPMV_ARR_SEND_IDX), want)
        assert spmv.spmv_get_info(s)["n_send"] == n
        spmv.spmv_set_schedule(s, schedule)
        c0 = gen.uniform_vector(A.n_rows, gen.rng_for(15, 0))
        C, send, recv = _exchange(s, x, hb, "f64", n, c0=c0)
        assert np.array_equal(send.view(np.uint64), oracle.pack(want, x).view(np.uint64))
        assert np.array_equal(recv, x[hb:])
        ref, den = oracle_ref(A, x, c0)
        assert_close(C, ref, den, FP64_TOL, "exchange cycle")
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32f64"])
def test_custom_list_bit_exact(prec):
    A, x = _irregular()
    hb = gen.halo_begin(A.n_cols)
    x = x.copy()
    x[5] = -0.0
    x[6] = np.inf
    if spmv.VEC_DTYPE[prec] == "float64":
        x[7] = np.array([0x7FF8DEADBEEF0001], dtype=np.uint64).view(np.float64)[0]
    rng = gen.rng_for(16, 0)
    idx = rng.integers(0, hb, size=70_001).astype(np.int32)
    idx[:4] = [5, 6, 7, 5]  # the special values, one of them twice
    a, s = _handles(A, hb, prec)
    try:
        spmv.spmv_set_send_list(s, idx)
        assert np.array_equal(spmv.spmv_export(s, spmv.SPMV_ARR_SEND_IDX), idx)
        _, send, _ = _exchange(s, x, hb, prec, idx.size)
        if spmv.VEC_DTYPE[prec] == "float64":
            want = oracle.pack(idx, x)
            assert np.array_equal(send.view(np.uint64), want.view(np.uint64))
        else:
            # B holds float32 values; the pack must return exactly them
            x32 = x.astype(np.float32)
            want = x32[idx]
            assert np.array_equal(send.view(np.uint32), want.view(np.uint32))
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


def test_products_unchanged_by_send_side():
    """The exchange product equals spmv_run's on the same inputs (bit for bit:
    same kernels, same plans, the pack only reads B)."""
    import torch

    A, x = _irregular()
    hb = gen.halo_begin(A.n_cols)
    a, s = _handles(A, hb)
    try:
        spmv.spmv_send_list_symmetric(s)
        n = spmv.spmv_get_info(s)["n_send"]
        C1, _, _ = _exchange(s, x, hb, "f64", n)
        B = to_dev(x, "f64")
        C2 = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
        spmv.spmv_run(s, B, C2)
        torch.cuda.synchronize()
        assert np.array_equal(C1, C2.cpu().numpy())
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


def test_lists_replaced_cleared_and_edges():
    A, x = _irregular()
    for hb in (0, 1, A.n_cols // 2, A.n_cols):
        a, s = _handles(A, hb)
        try:
            n = spmv.spmv_send_list_symmetric(s)
            assert np.array_equal(spmv.spmv_export(s, spmv.SPMV_ARR_SEND_IDX),
                                  oracle.send_list_symmetric(A.row_ptr, A.col_idx, hb))
            C, send, _ = _exchange(s, x, hb, "f64", n)
            if n:
                assert np.array_equal(send, oracle.pack(spmv.spmv_export(s, spmv.SPMV_ARR_SEND_IDX), x))
            ref, den = oracle_ref(A, x)
            assert_close(C, ref, den, FP64_TOL, f"exchange h={hb}")
            if hb > 0:
                # replace by a shorter list, then clear it
                spmv.spmv_set_send_list(s, np.array([hb - 1, 0, hb - 1], np.int32))
                _, send, _ = _exchange(s, x, hb, "f64", 3)
                assert send.tolist() == [x[hb - 1], x[0], x[hb - 1]]
            spmv.spmv_set_send_list(s, np.zeros(0, np.int32))
            assert spmv.spmv_get_info(s)["n_send"] == 0
            C, send, _ = _exchange(s, x, hb, "f64", 0)
            assert send.size == 0
            assert_close(C, ref, den, FP64_TOL, f"exchange without send h={hb}")
        finally:
            spmv.spmv_destroy(s)
            spmv.spmv_destroy(a)


def test_validation():
    import torch

    A, x = _irregular()
    hb = gen.halo_begin(A.n_cols)
    a, s = _handles(A, hb)
    try:
        for bad in ([hb], [-1], [0, 5, hb + 3]):
            with pytest.raises(spmv.SpmvError) as ei:
                spmv.spmv_set_send_list(s, np.array(bad, np.int32))
            assert ei.value.status == spmv.SPMV_ERR_INVALID_ARG and "outside" in ei.value.message
        lib = spmv.load()
        assert lib.spmv_set_send_list(spmv.ctypes.c_void_p(s.ptr), None, 3) == spmv.SPMV_ERR_INVALID_ARG
        assert lib.spmv_set_send_list(spmv.ctypes.c_void_p(s.ptr), None, -1) == spmv.SPMV_ERR_INVALID_ARG
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_set_send_list(a, np.array([0], np.int32))
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_send_list_symmetric(a)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        B = to_dev(x, "f64")
        C = to_dev(np.zeros(A.n_rows), "f64")
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_run_exchange(a, B, C)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        n = spmv.spmv_send_list_symmetric(s)
        # a send list but no send buffer
        st = lib.spmv_run_exchange(spmv.ctypes.c_void_p(s.ptr), spmv.ctypes.c_void_p(B.data_ptr()),
                                   spmv.ctypes.c_void_p(C.data_ptr()), None, None, None)
        assert st == spmv.SPMV_ERR_INVALID_ARG and "send_host" in spmv.spmv_last_error()
        # pageable send buffer rejected
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_run_exchange(s, B, C, None, torch.zeros(n, dtype=torch.float64))
        assert ei.value.status == spmv.SPMV_ERR_INVALID_ARG and "pinned" in ei.value.message
        with pytest.raises(ValueError):
            spmv.spmv_run_exchange(s, B, C, None, torch.zeros(n + 1, dtype=torch.float64).pin_memory())
        torch.cuda.synchronize()
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
    # with the flag, pageable buffers are accepted (and still correct)
    a, s = _handles(A, hb, flags=NOTUNE | spmv.SPMV_FLAG_ALLOW_PAGEABLE_HALO)
    try:
        n = spmv.spmv_send_list_symmetric(s)
        C, send, recv = _exchange(s, x, hb, "f64", n, pinned=False)
        assert np.array_equal(send, oracle.pack(spmv.spmv_export(s, spmv.SPMV_ARR_SEND_IDX), x))
        assert np.array_equal(recv, x[hb:])
        ref, den = oracle_ref(A, x)
        assert_close(C, ref, den, FP64_TOL, "pageable exchange with flag")
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


@pytest.mark.parametrize("P", [2, 3, 5])
def test_p_shares_exchange_cycle(P):
    """P nnz-balanced row shares of a symmetric matrix, each with its columns
    renumbered (owned first, then its halo): every share's exchange cycle on
    the GPU reproduces its rows of the full product bit for bit (integer
    data), and each share sends exactly what the others receive from it."""
    import test_partition as tp

    A = tp.integer_symmetric(30_000, gen.rng_for(951, P))
    x = gen.integer_vector(A.n_cols, gen.rng_for(951, 100 + P))
    full = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
    cuts = tp.shares(A.row_ptr, P)
    received, sent = {}, {}
    for p in range(P):
        r0, r1 = int(cuts[p]), int(cuts[p + 1])
        rp, col, val, h, halo = tp.share_matrix(A, r0, r1)
        Bp = np.concatenate([x[r0:r1], x[halo]])
        a = spmv.spmv_create_crs(rp, col, val, h + halo.size, flags=NOTUNE)
        s = spmv.spmv_split_local_nonlocal(a, h)
        try:
            n = spmv.spmv_send_list_symmetric(s)
            C, send, recv = _exchange(s, Bp, h, "f64", n)
            assert np.array_equal(recv, x[halo])
            assert np.array_equal(C, full[r0:r1])
            sent[p] = spmv.spmv_export(s, spmv.SPMV_ARR_SEND_IDX) + r0
            assert np.array_equal(send, x[sent[p]])
            received[p] = halo
        finally:
            spmv.spmv_destroy(s)
            spmv.spmv_destroy(a)
    for q in range(P):
        r0, r1 = int(cuts[q]), int(cuts[q + 1])
        wanted = np.unique(np.concatenate([received[p][(received[p] >= r0) & (received[p] < r1)]
                                           for p in range(P) if p != q] + [np.zeros(0, np.int64)]))
        assert np.array_equal(sent[q], wanted)


@pytest.mark.parametrize("local_plan", [None, dict(kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS, tile_items=2)],
                         ids=["default", "sorted"])
def test_phase_timing(local_plan):
    """Per-phase events: ordering under every schedule (the nonlocal part after
    the halo copy, everything after the call's start), and the error cases;
    with the local part in the default plan and in sorted blocks."""
    import torch

    A, x = _irregular()
    hb = gen.halo_begin(A.n_cols)
    a, s = _handles(A, hb)
    eps = 0.01  # ms of event-timestamp slack
    try:
        if local_plan:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, **local_plan)
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_phase_times(s)
        assert ei.value.status == spmv.SPMV_ERR_STATE
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_set_phase_timing(a, True)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        spmv.spmv_set_phase_timing(s, True)
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_phase_times(s)
        assert ei.value.status == spmv.SPMV_ERR_STATE
        n = spmv.spmv_send_list_symmetric(s)
        for schedule in MODES:
            spmv.spmv_set_schedule(s, schedule)
            for exchange in (False, True):
                if exchange:
                    _exchange(s, x, hb, "f64", n)
                else:
                    B = to_dev(x, "f64")
                    C = to_dev(np.zeros(A.n_rows), "f64")
                    spmv.spmv_run(s, B, C, torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory())
                    torch.cuda.synchronize()
                t = spmv.spmv_phase_times(s)
                assert t["copy"] and t["local"] and t["nonlocal"]
                assert (t["send"] is not None) == exchange
                for ph in t.values():
                    if ph:
                        assert -eps <= ph[0] <= ph[1] + eps
                assert t["copy"][1] <= t["nonlocal"][0] + eps
                merged = (schedule == spmv.SPMV_SCHEDULE_OVERLAP_MERGED and local_plan is not None
                          and local_plan["kernel"] == spmv.SPMV_KERNEL_SORTED_BLOCKS)
                if schedule == spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL or merged:
                    # the nonlocal part (merged: the last blocks over local and
                    # nonlocal entries) runs inside the local part's span
                    assert t["local"][0] <= t["nonlocal"][0] + eps
                    assert t["nonlocal"][1] <= t["local"][1] + eps
                else:
                    assert t["local"][1] <= t["nonlocal"][0] + eps
                if schedule == spmv.SPMV_SCHEDULE_SERIAL:
                    assert t["copy"][1] <= t["local"][0] + eps
                    if exchange:
                        assert t["send"][1] <= t["copy"][0] + eps
        spmv.spmv_set_phase_timing(s, False)
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_phase_times(s)
        assert ei.value.status == spmv.SPMV_ERR_STATE
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
