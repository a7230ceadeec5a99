"""The benchmark's algorithmic work formulas (the roofline numerators) and the
traffic lookup, checked by hand on small cases (CPU only)."""
import hashlib
import os

import bench


def test_lookup_bytes_by_hand():
    # E = 2: two targets, m = 10 - 1 = 9; E = 3: one target, m = 8.
    # per pair 4 L + 4 bytes; per (library, E in use) 8 m (E + 1) bytes.
    want = 2 * 2 * (40 + 4) + 2 * 8 * 9 * 3 + 2 * 1 * (40 + 4) + 2 * 8 * 8 * 4
    assert bench.lookup_bytes(2, 10, [2, 2, 3]) == want


def test_gram_flops_by_hand():
    # group 5..8, L = 20, Tp = 1: m = 20 - 4 - 1 = 15 ordered pairs m (m - 1),
    # 2 E_hi flops each
    assert bench.gram_flops(1, 20, 1, groups=((5, 8),)) == 2 * 8 * 15 * 14
    # a group cut at E_max uses the cut E_hi
    assert bench.gram_flops(1, 20, 1, groups=((5, 8),), E_max=6) == 2 * 6 * 15 * 14


def test_scan_ops_by_hand():
    # exact scan, E = 3, Tp = 0, L = 12: m = 10, 3E + 1 ops per ordered pair
    assert bench.scan_ops_exact(1, 12, [3], 0) == 10 * 9 * 10
    # an infeasible E (m - 1 < E + 1) adds nothing
    assert bench.scan_ops_exact(1, 6, [5], 0) == 0
    # grouped: one running key to E_hi plus one compare per E of the group
    assert bench.scan_ops_grouped(2, 12, ((1, 4),), 1) == 2 * 11 * 10 * (3 * 4 + 4)


def test_recorded_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "paper_2105_12301_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "lookup.hip").write_text("// kernel source\n")
    sha = hashlib.sha256(b"// kernel source\n").hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x.md").write_text(
        f"    bench-traffic: family=lookup sha256={sha} bytes_per_step=1.5e+09 workload=w\n"
        "    bench-traffic: family=lookup sha256=00 bytes_per_step=9e+09 workload=stale\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    tr = bench.recorded_traffic("lookup")
    assert tr == {"bytes_per_step": 1.5e9, "workload": "w", "source": "profiles/x.md"}
    (src / "lookup.hip").write_text("// changed\n")  # the counters no longer apply
    assert bench.recorded_traffic("lookup") is None
    assert bench.recorded_traffic("no_such_family") is None
    assert os.path.isdir(prof)
