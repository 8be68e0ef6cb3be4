"""Host logic of bench.py that runs without a GPU: the one-GPU guard, the
source hash that keys the committed PMC traffic, and the traffic lookup
(a line counts only while the hash of the kernel's sources matches)."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_source_hash_covers_the_shared_headers():
    b = _bench()
    h = hashlib.sha256()
    for path in (os.path.join(ROOT, "paper_2606_18588_amd", "csrc", "sx_render.hip"),
                 os.path.join(ROOT, "paper_2606_18588_amd", "csrc", "sx_internal.h"),
                 os.path.join(ROOT, "include", "splaxel.h")):
        with open(path, "rb") as f:
            h.update(f.read())
    assert b.source_sha("sx_render.hip") == h.hexdigest()[:16]
    assert b.source_sha("sx_render.hip") != b.source_sha("sx_sort.hip")


def test_traffic_lookup_needs_a_matching_hash(tmp_path, monkeypatch):
    b = _bench()
    k = "k_render_bwd<16, 16, false, false>"
    good = {"kernel": k, "source_sha": b.source_sha("sx_render.hip"),
            "hbm_bytes_per_launch": 1234.5}
    stale = {"kernel": "k_render<16, 16, false, false>", "source_sha": "0" * 16,
             "hbm_bytes_per_launch": 99.0}
    f = tmp_path / "traffic.txt"
    f.write_text("# header line\n" + json.dumps(good) + "\n" + json.dumps(stale) + "\n")
    monkeypatch.setattr(b, "PMC_FILE", str(f))
    assert b.pmc_traffic(k, "sx_render.hip") == 1234.5
    assert b.pmc_traffic("k_render<16, 16, false, false>", "sx_render.hip") is None
    assert b.pmc_traffic("no_such_kernel", "sx_render.hip") is None
    monkeypatch.setattr(b, "PMC_FILE", str(tmp_path / "missing.txt"))
    assert b.pmc_traffic(k, "sx_render.hip") is None
