"""Host-side parts of bench.py: the committed counter summaries are found
only for the workload, kernel sources and odd-kernel launch configuration
they were taken with."""
import glob
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summary_keys():
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        kv = {}
        for line in open(path):
            if line.startswith("traffic_") and ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        out.append(kv)
    return out


def test_every_summary_is_machine_readable():
    keys = _summary_keys()
    assert keys
    for kv in keys:
        for k in ("traffic_kernel", "traffic_workload", "traffic_bytes_per_launch",
                  "traffic_even_bytes_per_launch", "traffic_launch", "traffic_source_hash",
                  "traffic_odd_avg_us", "traffic_even_avg_us"):
            assert k in kv, k
        assert float(kv["traffic_bytes_per_launch"]) > 0
        assert float(kv["traffic_odd_avg_us"]) > 0


def test_recorded_profile_matches_workload_and_launch():
    """Values come back for the recorded workload and launch while the
    kernel sources hash to the recorded value, and never otherwise."""
    from paper_2408_06880_amd import kernel_source_hash
    current = kernel_source_hash()
    for kv in _summary_keys():
        launch = tuple(int(x) for x in kv["traffic_launch"].split("/"))
        prof = bench.recorded_profile(kv["traffic_workload"], launch)
        if kv["traffic_source_hash"] != current:      # summary older than the kernels
            assert prof is None
            continue
        assert prof["odd_bytes"] == float(kv["traffic_bytes_per_launch"])
        assert prof["even_bytes"] == float(kv["traffic_even_bytes_per_launch"])
        assert prof["odd_avg_us"] == float(kv["traffic_odd_avg_us"])
        assert prof["source"].startswith("profiles")
        other = launch[:4] + (launch[4] + 1,)
        assert bench.recorded_profile(kv["traffic_workload"], other) is None
    assert bench.recorded_profile("no such workload", (256, 1, 0, 1, 4)) is None
