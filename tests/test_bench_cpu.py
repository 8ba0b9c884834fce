"""Host-side checks of the benchmark script: the one-GPU limit and the committed counter
summaries it reads (no GPU needed)."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_summaries_have_what_the_benchmark_reads():
    sys.path.insert(0, ROOT)
    import bench

    for w, mode in (("surface_d25", "shared"), ("surface_d71", "shared"), ("random_batch", "batch")):
        p = json.load(open(os.path.join(ROOT, "profiles", f"pmc_{w}.json")))
        assert p["mode"] == mode and p["fetch_scale"] > 0 and p["write_scale"] > 0
        assert len(p["source_digest"]) == 16 and p["commands"]
        for k, v in p["kernels"].items():
            assert v["dispatches"] >= 1 and v["fetch_kib"] >= 0 and v["write_kib"] >= 0, (w, k)
        got = bench.load_pmc(w, mode, p.get("tile"))
        if p["source_digest"] == bench.kernel_source_digest():
            dom = {"surface_d25": "chain", "surface_d71": "segment", "random_batch": "batch"}[w]
            assert got.get(dom, 0) > 0
        else:
            assert got == {}
