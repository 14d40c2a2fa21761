"""Allocation failure injected at every step of setup: with
SPMV_FAULT_ALLOC_AFTER=n the n-th device allocation fails.  Each of
create, split, batch creation and the send list must then return
SPMV_ERR_ALLOC with a message naming the injection, leave no handle behind
and keep the process healthy (a later, successful run in the same process
gives the oracle's result).  Child processes, one at a time: the knob is read
once per process."""
from __future__ import annotations

import ast
import os
import subprocess
import sys

import pytest

from paper_1106_5908_amd import spmv

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import numpy as np
import oracle
from paper_1106_5908_amd import spmv
from workloads import gen

A, x = gen.workload_c3(N=20_000)
hb = gen.halo_begin(A.n_cols)
steps = []
def attempt(name, fn):
    try:
        r = fn()
        steps.append((name, "ok"))
        return r
    except spmv.SpmvError as e:
        steps.append((name, "err", e.status, "injected" in e.message))
        return None
a = attempt("create", lambda: spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols,
                                                    flags=spmv.SPMV_FLAG_NO_TUNE_CACHE))
s = attempt("split", lambda: spmv.spmv_split_local_nonlocal(a, hb)) if a is not None else None
if s is not None:
    attempt("send", lambda: spmv.spmv_send_list_symmetric(s))
b = attempt("batch", lambda: spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols)] * 3))
ok = None
if a is not None:
    import torch
    B = torch.from_numpy(x).to("cuda")
    C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    try:
        spmv.spmv_run(a, B, C)
        torch.cuda.synchronize()
        ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x)
        ok = bool(oracle.normalized_error(C.cpu().numpy(), ref, den).max() <= 1e-12)
    except spmv.SpmvError as e:
        ok = ("err", e.status, "injected" in e.message)
for h in (s, a, b):
    if h is not None:
        spmv.spmv_destroy(h)
print("STEPS", repr(steps), "RUN", repr(ok))
"""


def run_child(n: int):
    env = dict(os.environ)
    env["SPMV_FAULT_ALLOC_AFTER"] = str(n)
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("STEPS")][-1]
    steps_txt, run_txt = line[len("STEPS "):].split(" RUN ")
    return ast.literal_eval(steps_txt), ast.literal_eval(run_txt)


def test_allocation_failures_are_clean():
    seen_failure = False
    for n in (0, 1, 2, 3, 4, 6, 9, 13, 20, 30, 45):
        steps, run = run_child(n)
        for st in steps:
            if st[1] == "err":
                seen_failure = True
                assert st[2] == spmv.SPMV_ERR_ALLOC and st[3], (n, steps)
        if run is not None and run is not True:
            # the product itself may allocate tile tables: the same clean error
            assert run[0] == "err" and run[1] == spmv.SPMV_ERR_ALLOC and run[2], (n, run)
    assert seen_failure
    steps, run = run_child(10 ** 6)
    assert all(st[1] == "ok" for st in steps) and run is True, (steps, run)
