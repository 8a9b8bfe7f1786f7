"""Host-side checks of the autotuner's per-device file and of how bench.py
takes the counter-measured traffic from profiles/ (no GPU needed)."""
import json
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tuning_file_is_consistent():
    path = os.path.join(ROOT, "paper_2601_12713_amd", "tuning", "gfx950.json")
    with open(path) as f:
        t = json.load(f)
    best = t["best"]
    assert 1 <= best["blocks_per_cu"] <= 8
    assert best["split_bytes"] == 0 or 4096 <= best["split_bytes"] <= 65536
    assert best["use_graph"] == 1
    pts = t["points"]
    assert len(pts) >= 5, "the search covers at least five points"
    top = max(pts, key=lambda p: p["GBps"])
    assert (top["blocks_per_cu"], top["split_bytes"]) == (best["blocks_per_cu"], best["split_bytes"])
    for p in pts:
        assert p["ms"] > 0 and p["GBps"] > 0


def test_traffic_follows_the_sources(tmp_path, monkeypatch):
    import bench
    name = "digest_one_kernel.large-arrays"
    got = bench.traffic_from_profile(name, bench.DIGEST_SOURCES)
    pmc = os.path.join(ROOT, "profiles", name + ".pmc.txt")
    fields = dict(line.split(":", 1) for line in open(pmc) if ":" in line)
    if got is None:
        # the counters were taken on other sources: the line must say null, not a stale number
        pytest.skip("counter summary predates the current digest sources")
    assert got == int(fields["traffic_bytes_per_launch"].strip())
    # a changed source invalidates the figure
    repo = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "profiles"), repo / "profiles")
    for src in bench.DIGEST_SOURCES:
        dst = repo / src
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, src), dst)
    with open(repo / bench.DIGEST_SOURCES[0], "a") as f:
        f.write("\n// changed\n")
    monkeypatch.setattr(bench, "HERE", str(repo))
    assert bench.traffic_from_profile(name, bench.DIGEST_SOURCES) is None
