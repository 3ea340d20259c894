"""bench.py's counter-traffic records (profiles/traffic_*.json): each names the
kernel family, precision and source file it was measured on, and the bench
reports its bytes only for a run of that kernel, precision and source (CPU)."""
import glob
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


RECORDS = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")))


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p) for p in RECORDS])
def test_traffic_record_is_keyed_to_its_kernel(path):
    bench = load_bench()
    rec = json.load(open(path))
    for key in ("kernel_id", "precision", "kernel_source_file", "kernel_source_sha256",
                "fetch_kib_per_dispatch", "write_kib_per_dispatch", "fetch_scale", "write_scale",
                "command_fetch", "command_write"):
        assert key in rec, key
    # the commands run committed files only
    for cmd in (rec["command_fetch"], rec["command_write"]):
        assert "_work" not in cmd and "bench.py" in cmd
    workload = os.path.basename(path)[len("traffic_"):-len(".json")]
    kid, prec = rec["kernel_id"], rec["precision"]
    other_kernel = 4 if kid == 2 else 2
    other_prec = "fp64" if prec != "fp64" else "fp32"
    assert bench.measured_traffic(workload, other_kernel, prec) is None
    assert bench.measured_traffic(workload, kid, other_prec) is None
    current = rec["kernel_source_sha256"] == bench.kernel_source_digest(rec["kernel_source_file"])
    got = bench.measured_traffic(workload, kid, prec)
    if not current:
        assert got is None                  # a changed kernel reports no stale traffic
        pytest.skip("kernel source changed since the counters were taken")
    want = (rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] +
            rec["write_kib_per_dispatch"] * rec["write_scale"]) * 1024.0
    assert got == pytest.approx(want, rel=1e-12)
