"""Host logic of bench.py that the measurement depends on: which committed
counter summary a plan's traffic comes from, and the GPU kappa (Eq. (1)
analogue) computed from it.  Runs without a GPU."""
import json

import bench
from paper_1106_5908_amd import spmv

PLAN = {"kernel": 6, "tile_items": 2, "lanes": 32, "nontemporal": 1, "xcd_remap": 1,
        "block_kt": 0, "tiles_per_group": 1, "panels": 1}
NL = dict(PLAN, kernel=1, tile_items=4)


def _write(d, name, plan, workload, sha, traffic):
    (d / f"traffic_{name}.txt").write_text(json.dumps(
        {"kernel_sha": sha, "plan": plan, "pmc_workload": workload, "traffic_bytes": traffic}))


def test_traffic_needs_the_current_kernel_source_and_the_same_plan(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    sha = bench.kernel_hash()
    _write(tmp_path, "a", PLAN, "irregular8M", sha, 1.5e9)
    _write(tmp_path, "b", dict(PLAN, tile_items=4), "irregular8M", "0" * 16, 9.9e9)
    assert bench.read_traffic(PLAN, "irregular8M") == 1.5e9
    assert bench.read_traffic(PLAN, "27pt160") is None                   # other workload
    assert bench.read_traffic(dict(PLAN, tile_items=4), "irregular8M") is None  # stale source
    assert bench.read_traffic(dict(PLAN, xcd_remap=0), "irregular8M") is None   # other plan


def test_split_traffic_per_schedule(tmp_path, monkeypatch):
    """The ordered split needs both parts' plans to match; the merged tail
    runs no nonlocal kernel, so only its local plan and the schedule count."""
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    sha = bench.kernel_hash()
    merged = spmv.SPMV_SCHEDULE_OVERLAP_MERGED
    _write(tmp_path, "split", {"local": PLAN, "nonlocal": NL}, "irregular8M-split", sha, 1.8e9)
    _write(tmp_path, "merged", {"local": PLAN, "nonlocal": NL, "schedule": merged},
           "irregular8M-split", sha, 1.7e9)
    other_nl = dict(NL, tile_items=8)
    assert bench.read_traffic({"local": PLAN, "nonlocal": NL}, "irregular8M-split") == 1.8e9
    assert bench.read_traffic({"local": PLAN, "nonlocal": other_nl}, "irregular8M-split") is None
    assert bench.read_traffic({"local": PLAN, "nonlocal": other_nl, "schedule": merged},
                              "irregular8M-split") == 1.7e9
    assert bench.read_traffic({"local": dict(PLAN, tile_items=4), "nonlocal": NL,
                               "schedule": merged}, "irregular8M-split") is None


def test_kappa_is_extra_bytes_per_entry():
    nnz = 1_000_000
    flops = 2.0 * nnz
    model = 12.0 * nnz
    r = bench.traffic_report(model + 3.0 * nnz, model, flops)
    assert abs(r["kappa_gpu"] - 3.0) < 1e-12
    assert abs(r["traffic_over_model"] - 15.0 / 12.0) < 1e-12
    assert bench.traffic_report(None, model, flops) == {
        "traffic_bytes": None, "traffic_over_model": None, "kappa_gpu": None}
