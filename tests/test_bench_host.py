"""Host logic of bench.py: the kernel-source hash that guards the committed traffic record, the
record lookup, and the single-GPU guard."""
import json
import os
import shutil
import subprocess
import sys

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402

SRCS = ("nnplan.hip", "rollout.hpp", "philox.hpp")


def _tree(tmp_path):
    d = tmp_path / "paper_1904_06680_amd" / "csrc"
    d.mkdir(parents=True)
    for f in SRCS:
        shutil.copy(os.path.join(ROOT, "paper_1904_06680_amd", "csrc", f), d / f)
    return d


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    d = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.source_hash()
    p = d / "rollout.hpp"
    text = p.read_text()
    p.write_text("// a new line comment\n/* a block\n   comment */\n\n" + text + "\n// trailing\n")
    assert bench.source_hash() == h0
    p.write_text(text + "\nstatic constexpr int one_more_line = 1;\n")
    assert bench.source_hash() != h0


def test_traffic_record_only_for_the_recorded_sources(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"source_hash": "0123456789abcdef", "bytes_per_launch": 12345}
    (tmp_path / "profiles" / "rollout_c1_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_record("0123456789abcdef") == 12345
    assert bench.traffic_record("fedcba9876543210") is None
    (tmp_path / "profiles" / "rollout_c1_traffic.json").write_text("{not json")
    assert bench.traffic_record("0123456789abcdef") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_algorithmic_counts_closed_form():
    """C1 launch: 65536 x [51 x 3000 x 11 + 50 x (2 x 1344 + 66 + 75)] flops, and 3 more min/max
    operations per point test in the inclusive count."""
    w = (8, 32, 32, 2)
    f = bench.algorithmic_flops(65536, 50, 3000, w)
    assert f == 65536 * (51 * 3000 * 11 + 50 * (2 * 1344 + 66 + 75))
    assert bench.algorithmic_ops_with_minmax(65536, 50, 3000, w) == f + 65536 * 51 * 3000 * 3


def test_oracle_c0_plan_timing_leg():
    r = bench.oracle_c0_plan()
    assert r["kind"] == "oracle" and r["ms"] > 0 and r["cores"] >= 1
    assert abs(r["value"] - 1024 * 20 / (r["ms"] / 1e3)) <= 2e-3 * r["value"]     # ms is rounded


def test_executed_flops_bounds():
    """The executed work of a launch: all of the method's work when every point group is tested,
    the controller's share alone when none is, linear in between."""
    N, T, P, w = 65536, 50, 3000, (8, 32, 32, 2)
    full = bench.algorithmic_flops(N, T, P, w)
    assert bench.executed_flops(N, T, P, w, 1.0) == full
    ctrl = bench.executed_flops(N, T, P, w, 0.0)
    assert ctrl == float(N) * T * (bench.mlp_flops(w) + bench.FLOPS_STEP_OVERHEAD)
    half = bench.executed_flops(N, T, P, w, 0.5)
    assert abs(half - (full + ctrl) / 2) <= 1e-6 * full
