"""bench.py's contract on the host: more than one GPU is refused with a message,
and the HBM counter record is used only for the kernel sources it was taken from."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_is_tied_to_the_sources(tmp_path, monkeypatch):
    with open(bench.TV_TRAFFIC_RECORD) as fh:
        rec = json.load(fh)
    current = rec["sources_sha256"] == bench.tv_sources_digest()
    expected = rec["fetch_bytes"] + rec["write_bytes"] if current else None
    assert bench.tv_traffic(rec["tv_shape"], rec["voxels"]) == expected
    assert bench.tv_traffic(rec["tv_shape"] + 1, rec["voxels"]) is None
    stale = dict(rec, sources_sha256="0" * 64)
    p = tmp_path / "rec.json"
    p.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TV_TRAFFIC_RECORD", str(p))
    assert bench.tv_traffic(rec["tv_shape"], rec["voxels"]) is None


def test_unknown_extra_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--extras", "differentiable,nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "nope" in r.stderr
    assert r.stdout.strip() == ""
