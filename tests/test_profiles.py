"""The committed HBM-traffic figures (profiles/traffic.json) name the kernel sources they
were measured on: the benchmark reports roofline.traffic only while the kernel's source hash
still matches, and null once the kernel has changed since its counters were taken."""
import json
import os

import bench
from paper_2508_11443_amd import counters

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_file_is_reported_only_for_unchanged_kernels():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        d = json.load(f)
    assert set(d) == set(counters.KERNELS)
    for name, v in d.items():
        assert v["source"] == counters.KERNELS[name][1] == bench.KERNEL_SRC[name]
        assert v["hbm_bytes_per_launch"] == v["fetch_bytes_per_launch"] + v["write_bytes_per_launch"]
        fresh = v["source_sha"] == counters.src_sha(v["source"])
        assert bench.load_traffic(name) == (v["hbm_bytes_per_launch"] if fresh else None), name
