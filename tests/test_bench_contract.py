"""CPU checks of the benchmark script's contract: one GPU only, and the
calibrated traffic table belongs to the kernel source it ships with (a
kernel edit needs new FETCH_SIZE / WRITE_SIZE runs; until then bench.py
reports traffic as null)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_table_is_keyed_by_kernel_source():
    # entries are keyed by the sha256 of the kernel source they were measured
    # on; a launch of another source finds none and reports traffic null
    sys.path.insert(0, ROOT)
    import bench
    for sha, table in bench.TRAFFIC.items():
        assert len(sha) == 64 and all(c in "0123456789abcdef" for c in sha)
        for key, entries in table.items():
            assert entries, key
            for t in entries:
                assert t["workgroups"] > 0 and t["read_bytes"] > 0 and t["write_bytes"] > 0, key


def test_traffic_entry_matches_shape_and_source():
    sys.path.insert(0, ROOT)
    import bench
    for sha, table in bench.TRAFFIC.items():
        _check_entries(bench, sha, table)
    assert bench.traffic_entry(bench.kernel_sha() + "x", "c5/fp64", 3072) is None


def _check_entries(bench, sha, table):
    for key, entries in table.items():
        for e in entries:
            assert bench.traffic_entry(sha, key, e["workgroups"]) is e
        # a launch shape that was not measured, another source, another workload
        assert bench.traffic_entry(sha, key, 1 + max(e["workgroups"] for e in entries)) is None
        assert bench.traffic_entry("0" * 64, key, entries[0]["workgroups"]) is None
    assert bench.traffic_entry(sha, "no/such", 760) is None
