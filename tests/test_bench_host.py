"""Host-side logic of bench.py (no GPU): the one-GPU contract, the
algorithmic byte models the rooflines divide by, and the traffic summary's
link to the walk sources."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_walk_bytes_model():
    # per hop (the start edge included): 4 random 64 B sectors for a biased
    # pick, 3 for a uniform one, and 12 B of output; per walk its length and
    # first node (8 B); padding slots are not counted
    S = bench.SECTOR
    assert bench.walk_bytes(1, 0, "uniform") == 8
    assert bench.walk_bytes(2, 5, "linear") == 5 * (4 * S + 12) + 16
    assert bench.walk_bytes(0, 7, "uniform") == 7 * (3 * S + 12)
    # the stream workload's linear hops: 268 B each
    assert bench.walk_bytes(0, 1, "linear") == 268


def test_ingest_bytes_models():
    # incremental: 16 B read per input record, 80 B per kept record (sort
    # pass, timestamp view and group start, node view and group record),
    # 4 B per evicted record, 96 B per touched node record
    assert bench.ingest_bytes(10, 0, 0, 0) == 160
    assert bench.ingest_bytes(0, 1, 0, 0) == 80
    assert bench.ingest_bytes(0, 0, 3, 2) == 12 + 192
    # rebuild: batch read, one sort pass, 28 B per window record read and
    # written, 4 B per node
    assert bench.rebuild_bytes(1, 2, 3, 5) == 16 + 32 + 28 * 5 + 20


def test_traffic_summary_is_tied_to_the_walk_sources(tmp_path, monkeypatch):
    # the committed summary counts only while the walk sources hash to its
    # value: a changed hash turns traffic into None
    with open(bench.TRAFFIC_FILES["single"]) as fh:
        head, tail = fh.read().split("\n---\n", 1)
    rec = json.loads(head)
    assert rec["fetch_bytes"] > 0 and rec["write_bytes"] > 0
    assert set(rec) >= {"kernel", "workload", "fetch_scale", "write_scale", "source_sha256"}
    t = bench.measured_traffic("single")
    assert t is None or t == rec["fetch_bytes"] + rec["write_bytes"]
    assert bench.measured_traffic("mixed") is None
    fake = tmp_path / "traffic.txt"
    rec["source_sha256"] = "0" * 64
    fake.write_text(json.dumps(rec) + "\n---\n" + tail)
    monkeypatch.setitem(bench.TRAFFIC_FILES, "single", str(fake))
    assert bench.measured_traffic("single") is None
