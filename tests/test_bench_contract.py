"""Host-side parts of bench.py that need no GPU: the one-GPU refusal, the
counter-summary guard that keeps `roofline.traffic` null once the kernel
sources differ from the ones the counters were taken on, and the committed
summaries naming files that exist."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _summary(tmp_path, src_text, sha=None):
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "k.hip").write_text(src_text)
    digest = sha or hashlib.sha256(src_text.encode()).hexdigest()
    summ = dict(sources=["k.hip"], sources_sha256=digest, fetch_kib_per_launch=100.0,
                fetch_scale=2.0, write_kib_per_launch=50.0, write_scale=1.0, command="cmd")
    (tmp_path / "profiles" / "k_pmc.json").write_text(json.dumps(summ))


def test_traffic_only_while_sources_match(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _summary(tmp_path, "kernel v1")
    got, src = bench.pmc_traffic(1, name="k_pmc.json")
    assert got == (100.0 * 2.0 + 50.0 * 1.0) * 1024.0 and src == "cmd"
    (tmp_path / "k.hip").write_text("kernel v2")           # a source changed since
    got, why = bench.pmc_traffic(1, name="k_pmc.json")
    assert got is None and "changed" in why
    got, why = bench.pmc_traffic(1, name="missing.json")
    assert got is None


def test_committed_summaries_name_existing_sources():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if not name.endswith("_pmc.json"):
            continue
        with open(os.path.join(ROOT, "profiles", name)) as f:
            summ = json.load(f)
        assert summ["sources"], name
        for s in summ["sources"]:
            assert os.path.exists(os.path.join(ROOT, s)), (name, s)
        assert summ["fetch_scale"] > 0 and summ["write_scale"] > 0, name
