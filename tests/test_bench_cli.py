"""bench.py's command line on a machine without a GPU: it parses, documents
its options, and refuses more than one GPU before touching any device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_help_lists_the_options():
    r = run("--help")
    assert r.returncode == 0, r.stderr
    for opt in ("--gpus", "--steps", "--warmup", "--settle-ms", "--only", "--sweep", "--no-cpu"):
        assert opt in r.stdout


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_counter_record_is_used_only_on_its_source(tmp_path, monkeypatch):
    """The HBM-traffic and VALU figures come from the committed counter record
    only while its source digest matches the library sources."""
    import json
    b = _bench_module()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"src_digest": b.src_digest(), "bytes_per_launch": 2.0e8, "valu_insts_per_launch": 3.0e7,
           "lanes_active": 0.8, "summary": "profiles/x.md"}
    (prof / "traffic_k.json").write_text(json.dumps(rec))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setattr(b, "src_digest", lambda: rec["src_digest"])
    assert b.traffic_for("k") == 2.0e8
    v = b.valu_issue_for("k", 0.1)
    assert v["insts_per_launch"] == 3.0e7
    assert abs(v["frac"] - 3.0e7 / 1e-4 / (256 * 4 * 2.4e9 / 4)) < 1e-12
    monkeypatch.setattr(b, "src_digest", lambda: "another source")
    assert b.traffic_for("k") is None and b.valu_issue_for("k", 0.1) is None
    assert b.traffic_for("missing") is None
