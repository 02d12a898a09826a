"""Host-side logic of bench.py (no GPU): a counter summary is used only
while it was taken on the current sources of the batched kernels, and a
request for more than one GPU is refused with a message."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_source_hash_covers_every_schedule_source(tmp_path):
    files = []
    for i in range(3):
        p = tmp_path / f"f{i}"
        p.write_bytes(b"x%d" % i)
        files.append(str(p))
    base = bench._source_hash(files)
    for p in files:
        old = open(p, "rb").read()
        open(p, "wb").write(old + b" ")
        assert bench._source_hash(files) != base, p
        open(p, "wb").write(old)
    assert bench._source_hash(files) == base
    names = {os.path.basename(p) for p in bench.KERNEL_SOURCES}
    assert names == {"batch.hip", "hot_dense.hip", "ahpp_internal.h", "graph_build.hip"}


@pytest.mark.parametrize("kind", sorted(bench.TRAFFIC_FILES))
def test_committed_summaries_are_consistent(kind):
    """Each committed summary names its kernel and scales both counters by a
    copy of known size; the bench uses it only while its source hash holds."""
    d = json.load(open(bench.TRAFFIC_FILES[kind]))
    assert d["kernel"] == kind and len(d["source_sha256_16"]) == 16
    cal = d["copy_calibration"]
    assert cal["fetch_scale"] == pytest.approx(cal["bytes"] / 1024 / cal["fetch_kib_raw"])
    assert cal["write_scale"] == pytest.approx(cal["bytes"] / 1024 / cal["write_kib_raw"])
    want = (d["fetch_kib_per_dispatch_raw"] * cal["fetch_scale"] + d["write_kib_per_dispatch_raw"] *
            cal["write_scale"]) * 1024
    assert d["bytes_per_launch"] == pytest.approx(want)
    current = d["source_sha256_16"] == bench._source_hash(bench.KERNEL_SOURCES)
    assert bench._traffic(kind) == (d["bytes_per_launch"] if current else None)


def test_stale_summary_is_ignored(tmp_path, monkeypatch):
    kind = sorted(bench.TRAFFIC_FILES)[0]
    d = json.load(open(bench.TRAFFIC_FILES[kind]))
    d["source_sha256_16"] = "0" * 16
    p = tmp_path / "t.json"
    p.write_text(json.dumps(d))
    monkeypatch.setitem(bench.TRAFFIC_FILES, kind, str(p))
    assert bench._traffic(kind) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
