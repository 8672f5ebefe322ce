"""bench.py's host-side bookkeeping (no GPU): the algorithmic byte model and
the lookup of counter traffic by kernel source and launch shape."""
import json
import os

import bench


def test_algorithmic_bytes_per_link_update():
    # one read of every link of the lattice and one write of the updated
    # half-direction: (2D + 1) S per link update, S the stored link
    assert bench.BYTES_PER_LINK == {0: 144, 1: 72, 2: 48, 3: 96}
    for name, (ext, prec, _beta) in bench.WORKLOADS.items():
        D = len(ext)
        assert (2 * D + 1) * bench.BYTES_PER_LINK[prec] in (1296, 648, 432, 864), name


def test_traffic_lookup_follows_source_hash_and_launch_shape():
    seen = 0
    for name in bench.WORKLOADS:
        path = os.path.join(bench.PROFILES, f"update_kernel_{name}_pmc.json")
        if not os.path.exists(path):
            assert bench.measured_traffic(name, (256, 0, 2)) is None
            continue
        rec = json.load(open(path))
        current = rec["kernel_source_hash"] == bench.kernel_source_hash()
        for key, entry in rec["by_launch"].items():
            shape = tuple(int(v) for v in key.split(","))
            got = bench.measured_traffic(name, shape)
            assert got == (entry["hbm_bytes_per_launch"] if current else None), (name, key)
            # the record is the one its profiling command asked for
            assert key in entry["launch_cmd"], (name, key)
            seen += 1
        # a shape no counter run covers reports no traffic
        assert bench.measured_traffic(name, (64, 31, 9)) is None
    assert seen > 0


def test_small_configs_are_the_papers_runs():
    c = bench.SMALL_CONFIGS
    assert c["config1_4^4_cold"] == ((4, 4, 4, 4), 1, 0, True, 6.0, 20)
    assert c["config3_2x24^3x8_hot"][:3] == ((24, 24, 24, 8), 2, 0xF)
    assert {v[4] for k, v in c.items() if k.startswith("config2a")} == {5.7, 6.0}
