"""The committed HBM-traffic figures (profiles/traffic.json) were measured on the kernel
sources in the tree: the benchmark reports roofline.traffic only while each kernel's source
hash matches, so a kernel changed after its counters were taken shows up here."""
import json
import os

from paper_2508_11443_amd import counters

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_file_matches_the_sources():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        d = json.load(f)
    assert set(d) == set(counters.KERNELS)
    for name, v in d.items():
        assert v["source"] == counters.KERNELS[name][1]
        assert v["source_sha"] == counters.src_sha(v["source"]), name
        assert v["hbm_bytes_per_launch"] == v["fetch_bytes_per_launch"] + v["write_bytes_per_launch"]
