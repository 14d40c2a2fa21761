"""The C interface without a GPU: the library loads, exports every entry
point the header declares, and rejects invalid input before touching the
device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1106_5908_amd import spmv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmv.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spmv_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = spmv.load()
    names = declared_symbols()
    assert "spmv_create_crs" in names and "spmv_run_block" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(spmv.EXPORTED) == names


def _create(rp, ci, v, n_cols, base=0, prec=0, n_rows=None, nnz=None):
    lib = spmv.load()
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci, np.int32)
    v = np.ascontiguousarray(v, np.float64)
    out = ctypes.c_void_p(123)
    st = lib.spmv_create_crs(rp.size - 1 if n_rows is None else n_rows, n_cols,
                             ci.size if nnz is None else nnz, rp.ctypes.data,
                             ci.ctypes.data if ci.size else None, v.ctypes.data if v.size else None,
                             base, prec, 0, ctypes.byref(out))
    return st, out.value, spmv.spmv_last_error()


GOOD = ([0, 2, 3], [0, 2, 1], [1.0, 2.0, 3.0], 3)


@pytest.mark.parametrize("case,status,msg", [
    (dict(rp=[1, 2, 3]), spmv.SPMV_ERR_INVALID_MATRIX, "row_ptr[0]"),
    (dict(rp=[0, 2, 4]), spmv.SPMV_ERR_INVALID_MATRIX, "row_ptr[2]"),
    (dict(rp=[0, 3, 3], ci=[0, 2, 1]), None, None),
    (dict(rp=[0, 4, 3], ci=[0, 2, 1]), spmv.SPMV_ERR_INVALID_MATRIX, "decreases at index 2"),
    (dict(ci=[0, 3, 1]), spmv.SPMV_ERR_INVALID_MATRIX, "col_idx[1]"),
    (dict(ci=[0, -1, 1]), spmv.SPMV_ERR_INVALID_MATRIX, "col_idx[1]"),
    (dict(base=2), spmv.SPMV_ERR_INVALID_ARG, "index_base"),
    (dict(prec=9), spmv.SPMV_ERR_INVALID_ARG, "precision"),
    (dict(n_cols=-1), spmv.SPMV_ERR_INVALID_ARG, "negative"),
    (dict(nnz=2 ** 31), spmv.SPMV_ERR_INVALID_ARG, "int32"),
    (dict(base=1), spmv.SPMV_ERR_INVALID_MATRIX, "row_ptr[0]"),
])
def test_create_rejects_invalid(case, status, msg):
    rp, ci, v, n_cols = GOOD
    rp = case.get("rp", rp)
    ci = case.get("ci", ci)
    n_cols = case.get("n_cols", n_cols)
    st, out, err = _create(rp, ci, v, n_cols, base=case.get("base", 0), prec=case.get("prec", 0),
                           nnz=case.get("nnz"))
    if status is None:
        # a non-decreasing row_ptr with a trailing empty row is valid; without a
        # GPU the call then fails only at the device stage
        assert st in (spmv.SPMV_OK, spmv.SPMV_ERR_HIP, spmv.SPMV_ERR_ALLOC), err
        if st == spmv.SPMV_OK:
            spmv.load().spmv_destroy(ctypes.c_void_p(out))
        return
    assert st == status, (st, err)
    assert msg in err
    assert out is None


def test_one_based_columns_checked_against_shifted_range():
    # with index_base = 1 columns must lie in [1, n_cols]
    st, _, err = _create([1, 3, 4], [1, 4, 2], [1.0, 2.0, 3.0], 3, base=1)
    assert st == spmv.SPMV_ERR_INVALID_MATRIX and "col_idx[1]" in err


def test_null_arguments():
    lib = spmv.load()
    assert lib.spmv_create_crs(1, 1, 1, None, None, None, 0, 0, 0, None) == spmv.SPMV_ERR_INVALID_ARG
    rp = np.array([0, 1], np.int32)
    out = ctypes.c_void_p()
    assert lib.spmv_create_crs(1, 1, 1, rp.ctypes.data, None, None, 0, 0, 0,
                               ctypes.byref(out)) == spmv.SPMV_ERR_INVALID_ARG
    assert "null" in spmv.spmv_last_error()
    assert lib.spmv_run(None, None, None, None, None) == spmv.SPMV_ERR_INVALID_ARG
    assert lib.spmv_run_block(None, 1, None, 1, None, 1, None) == spmv.SPMV_ERR_INVALID_ARG
    assert lib.spmv_split_local_nonlocal(None, 0, ctypes.byref(out)) == spmv.SPMV_ERR_INVALID_ARG


def test_destroy_null_and_foreign():
    lib = spmv.load()
    assert lib.spmv_destroy(None) == spmv.SPMV_OK
    fake = (ctypes.c_char * 64)()
    assert lib.spmv_destroy(ctypes.cast(fake, ctypes.c_void_p)) == spmv.SPMV_ERR_STATE
    assert lib.spmv_run(ctypes.cast(fake, ctypes.c_void_p), None, None, None, None) == spmv.SPMV_ERR_STATE


def test_batch_validation_names_member():
    lib = spmv.load()
    rps = [np.array([0, 1], np.int32), np.array([0, 1], np.int32)]
    cis = [np.array([0], np.int32), np.array([5], np.int32)]
    vs = [np.array([1.0]), np.array([2.0])]
    arr = lambda xs: (ctypes.c_void_p * 2)(*[x.ctypes.data for x in xs])  # noqa: E731
    n = np.array([1, 1], np.int64)
    out = ctypes.c_void_p()
    st = lib.spmv_create_batch(2, n.ctypes.data, n.ctypes.data, n.ctypes.data, arr(rps), arr(cis),
                               arr(vs), 0, 0, 0, ctypes.byref(out))
    assert st == spmv.SPMV_ERR_INVALID_MATRIX
    assert "member 1" in spmv.spmv_last_error()
    assert lib.spmv_create_batch(0, None, None, None, None, None, None, 0, 0, 0,
                                 ctypes.byref(out)) == spmv.SPMV_ERR_INVALID_ARG


def test_probe_argument_checks():
    lib = spmv.load()
    assert lib.spmv_probe_spin(-1, None) == spmv.SPMV_ERR_INVALID_ARG
    assert lib.spmv_probe_copy(None, None, 5, None) == spmv.SPMV_ERR_INVALID_ARG
    assert lib.spmv_probe_triad(None, None, None, 1.0, -1, None) == spmv.SPMV_ERR_INVALID_ARG
    assert lib.spmv_probe_gather(None, 10, 3, None, 0, 1, None, 0, None) == spmv.SPMV_ERR_INVALID_ARG
    assert lib.spmv_probe_gather(None, 10, 1, None, 5, 1, None, 0, None) == spmv.SPMV_ERR_INVALID_ARG
    assert lib.spmv_probe_gather_sums_needed(100, 3) == -1
    assert lib.spmv_probe_gather_sums_needed(0, 1) == 0
    assert lib.spmv_probe_gather_sums_needed(2049, 1) == 2
    assert lib.spmv_probe_gather_sums_needed(2049, 16) == 9


def test_errors_are_per_thread():
    """Failing calls from many threads at once: each thread reads its own
    message (spmv_last_error is thread-local) and gets its own status."""
    import threading

    lib = spmv.load()
    cases = [(dict(rp=[1, 2, 3]), "row_ptr[0]"), (dict(ci=[0, 3, 1]), "col_idx[1]"),
             (dict(base=2), "index_base"), (dict(prec=9), "precision"),
             (dict(n_cols=-1), "negative"), (dict(rp=[0, 4, 3], ci=[0, 2, 1]), "decreases")]
    results = {}
    barrier = threading.Barrier(len(cases) * 4)

    def worker(i, case, msg):
        barrier.wait()
        for _ in range(200):
            rp, ci, v, n_cols = GOOD
            st, out, err = _create(case.get("rp", rp), case.get("ci", ci), v, case.get("n_cols", n_cols),
                                   base=case.get("base", 0), prec=case.get("prec", 0))
            if st == spmv.SPMV_OK or msg not in err or out is not None:
                results[i] = (st, err)
                return
        results[i] = None

    threads = [threading.Thread(target=worker, args=(4 * j + r, c, m))
               for j, (c, m) in enumerate(cases) for r in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert all(v is None for v in results.values()), results
    assert lib is spmv.load()
