"""Host logic of bench.py that needs no GPU: the one-GPU guard, the mode
dispatch, and the rule that the HBM traffic recorded with rocprofv3 is
reported only while the sweep source it was measured on is unchanged."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_unknown_mode_is_refused():
    r = _run("--mode", "no-such-mode")
    assert r.returncode != 0
    assert "unknown mode" in (r.stdout + r.stderr)


@pytest.fixture
def bench_module():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def _fake_tree(tmp_path, sha, source=b"// sweep\n"):
    src = tmp_path / "paper_2005_10431_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "stencil.hip").write_bytes(source)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps({"cfg4_fp64_sweep": {"bytes_per_launch": 123.0,
                                                                        "source_sha": sha}}))


def test_traffic_is_reported_only_for_the_measured_source(bench_module, tmp_path, monkeypatch):
    source = b"// sweep\n"
    sha = hashlib.sha256(source).hexdigest()[:16]
    _fake_tree(tmp_path, sha, source)
    monkeypatch.setattr(bench_module, "ROOT", str(tmp_path))
    assert bench_module.traffic_record("cfg4_fp64_sweep") == 123.0
    assert bench_module.traffic_record("cfg2_fp64_sweep") is None
    # the source changed since the counters were taken: no traffic figure
    (tmp_path / "paper_2005_10431_amd" / "csrc" / "stencil.hip").write_bytes(source + b"// edited\n")
    assert bench_module.traffic_record("cfg4_fp64_sweep") is None


def test_committed_traffic_record_names_its_summary(bench_module):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, r in rec.items():
        assert r["summary"].startswith("profiles/") and os.path.exists(os.path.join(ROOT, r["summary"]))
        assert r["bytes_per_launch"] >= r["algorithmic_bytes"]
