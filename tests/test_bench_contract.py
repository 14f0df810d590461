"""Host-side parts of the benchmark's contract that need no GPU: more than
one GPU is refused with a message (this library runs on one), and the
counter-measured traffic figures are only used for the sources they were
taken on."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout == ""


def test_traffic_figures_follow_the_sources(tmp_path, monkeypatch):
    b = _bench()
    with open(b.TRAFFIC_FILE) as f:
        d = json.load(f)
    # keyed to these sources: the figure is used; for other sources or
    # another workload it is not
    ok = d.get("source_sha256") == b.library_source_sha()
    t = b.measured_traffic("k_backproject", "uterus256")
    assert (t is not None) == ok
    if ok:
        e = d["kernels"]["k_backproject"]
        assert t == float(e["fetch_bytes"]) + float(e["write_bytes"])
    assert b.measured_traffic("k_backproject", "batched") is None
    stale = dict(d, source_sha256="0" * 64)
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(stale))
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(p))
    assert b.measured_traffic("k_backproject", "uterus256") is None
