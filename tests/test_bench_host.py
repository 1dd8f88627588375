"""Host checks of bench.py's bookkeeping: a stored HBM counter reading is
used only for the launch it was taken on (same kernel sources, tile side
and launched workgroups)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _record(workload):
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json")) as f:
        return json.load(f)


def test_stored_traffic_needs_the_measured_launch():
    ops = {"c1": "accum", "c2": "ca2", "c3": "ca3", "c4": "hash"}
    for w, op in ops.items():
        rec = _record(w)
        info = {"rho": rec["rho"], "launched_wgs": rec.get("launched_wgs", 0)}
        want = rec["hbm_bytes_per_launch"] if rec["kernel_sha"] == bench.kernel_sha(op) else None
        assert bench.stored_traffic(w, op, info) == want
        # another tile side, or another workgroup count where one is recorded
        assert bench.stored_traffic(w, op, dict(info, rho=info["rho"] * 2)) is None
        if "launched_wgs" in rec:
            assert bench.stored_traffic(w, op, dict(info, launched_wgs=info["launched_wgs"] + 1)) is None


def test_stored_traffic_absent_workload():
    assert bench.stored_traffic("c9", "ca2", {"rho": 1024, "launched_wgs": 1}) is None


def test_each_record_names_its_tile_in_the_kernel():
    # the kernel's first (automata) or second (per-element) template argument is rho
    for w in ("c1", "c2", "c3", "c4"):
        rec = _record(w)
        targs = [t.strip() for t in rec["kernel"].split("<", 1)[1].split(">")[0].split(",")]
        rho = int(targs[1]) if "k_point" in rec["kernel"] else int(targs[0])
        assert rho == rec["rho"], w
