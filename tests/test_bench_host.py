"""Host-side logic of bench.py (no GPU): the HBM-traffic figures it reports are
taken from the committed counter summary only while the kernel sources still
hash to the value stored with the counters, and the command line refuses more
than one GPU."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summary(tmp_path, srcs, digest, fwd=123456, vjp=654321):
    p = tmp_path / "traffic.txt"
    lines = ["# test summary", f"traffic_bytes.forward = {fwd}", f"traffic_bytes.ift_vjp = {vjp}",
             "kernel sources these counters were taken from:"]
    lines += [f"  {s}" for s in srcs]
    lines.append(f"sources_sha256 = {digest}")
    p.write_text("\n".join(lines) + "\n")
    return str(p)


def _digest(srcs):
    h = hashlib.sha256()
    for s in srcs:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    return h.hexdigest()


def test_traffic_read_when_sources_match(tmp_path, monkeypatch):
    srcs = ["paper_2607_24959_amd/csrc/cs_small.hpp", "paper_2607_24959_amd/csrc/cs_device.hpp"]
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, srcs, _digest(srcs)))
    assert bench.measured_traffic("forward") == 123456
    assert bench.measured_traffic("ift_vjp") == 654321
    assert bench.measured_traffic("missing") is None


def test_traffic_dropped_when_sources_changed(tmp_path, monkeypatch):
    srcs = ["paper_2607_24959_amd/csrc/cs_small.hpp", "paper_2607_24959_amd/csrc/cs_device.hpp"]
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, srcs, "0" * 64))
    assert bench.measured_traffic("forward") is None
    # no source list at all: nothing can be checked, so nothing is reported
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, [], _digest([])))
    assert bench.measured_traffic("forward") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.txt"))
    assert bench.measured_traffic("forward") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
