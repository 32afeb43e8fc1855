"""Host logic of bench.py (no GPU): the search that matches an opening
parameter along a run, and the lookup of committed traffic records."""
import json
import os

import pytest

import bench


def _run_of(limit, power=2.0):
    """A synthetic error run: the largest p99 along the run grows as x^power
    and reaches the 1e-3 target at x = limit."""
    calls = []

    def run(x):
        calls.append(x)
        return dict(max=bench.TARGET_P99 * (x / limit) ** power, builds=0)
    return run, calls


@pytest.mark.parametrize("limit,power", [(0.08, 2.0), (0.05, 3.0), (0.031, 1.0)])
def test_match_along_run_finds_the_largest_matched_value(limit, power):
    run, calls = _run_of(limit, power)
    x, r = bench.match_along_run("synthetic", run, 0.1, 2.0, bench.THETA_FLOOR, guess=0.09)
    assert r["max"] <= bench.TARGET_P99
    assert limit * (1 - 0.03) <= x <= limit
    assert len(calls) <= 6


def test_match_along_run_keeps_x0_when_it_already_meets_the_target():
    run, _ = _run_of(0.2)
    x, r = bench.match_along_run("synthetic", run, 0.1, 2.0, bench.THETA_FLOOR)
    assert x == 0.1 and r["max"] <= bench.TARGET_P99


def test_match_along_run_raises_when_the_floor_misses():
    run, calls = _run_of(0.001)             # even the floor (0.02) is far above the target
    with pytest.raises(RuntimeError):
        bench.match_along_run("synthetic", run, 0.1, 2.0, bench.THETA_FLOOR)
    assert min(calls) == bench.THETA_FLOOR


def test_traffic_record_lookup(tmp_path, monkeypatch):
    """A record counts only for its workload, group size, theta and force-kernel
    source; anything else gives null."""
    digest = bench.force_source_digest()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1907_02289_amd" / "csrc").mkdir(parents=True)
    for f in ("bh_force.hip", "bh_walk.hip"):
        src = os.path.join(bench.ROOT, "paper_1907_02289_amd", "csrc", f)
        (tmp_path / "paper_1907_02289_amd" / "csrc" / f).write_bytes(open(src, "rb").read())
    rec = dict(workload="ring16_kdk1+2", n_group=384, theta=0.0842, kernel_source_sha256_16=digest,
               hbm_bytes_per_launch=123.0)
    (tmp_path / "profiles" / "force_kernel_traffic.json").write_text(json.dumps([rec]))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("ring16_kdk1+2", 384, 0.0842) == 123.0
    assert bench.measured_traffic("ring16_kdk1+2", 256, 0.0842) is None
    assert bench.measured_traffic("ring16_kdk1+2", 384, 0.0843) is None
    assert bench.measured_traffic("ring16_kdk5+20", 384, 0.0842) is None
    (tmp_path / "paper_1907_02289_amd" / "csrc" / "bh_walk.hip").write_bytes(b"// changed work order\n")
    assert bench.measured_traffic("ring16_kdk1+2", 384, 0.0842) is None


def test_committed_traffic_record_matches_the_force_kernel_source():
    """The committed record was taken on the current force-kernel and walk
    sources (a changed kernel or work order needs new counter runs)."""
    recs = json.load(open(os.path.join(bench.ROOT, "profiles", "force_kernel_traffic.json")))
    assert any(r["kernel_source_sha256_16"] == bench.force_source_digest() for r in recs)
