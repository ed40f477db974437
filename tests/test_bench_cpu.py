"""Host-side plumbing of bench.py (no GPU): the recorded HBM traffic is used
only while the hashed kernel sources are unchanged and the workload matches,
and a multi-GPU request is refused with an explanation."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_source_sha_tracks_every_file(tmp_path):
    a, b = tmp_path / "a.hip", tmp_path / "b.h"
    a.write_text("kernel one\n")
    b.write_text("header\n")
    h0 = bench.kernel_source_sha([str(a), str(b)])
    assert h0 == bench.kernel_source_sha([str(a), str(b)]) and len(h0) == 16
    b.write_text("header changed\n")
    assert bench.kernel_source_sha([str(a), str(b)]) != h0


def test_recorded_traffic_only_for_matching_sources_and_workload():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, sources, wl in [("lse_partial_fp32<64,4>", None, "gmm16k_d64_fp32"),
                             ("pcost_lse", bench.PCOST_SOURCES, "pcost_4i_d47")]:
        r = rec[key]
        got = bench.recorded_traffic(key, wl, sources)
        if r["kernel_sha256_16"] == bench.kernel_source_sha(sources):
            assert got == float(r["fetch_bytes_per_launch"] + r["write_bytes_per_launch"])
        else:
            assert got is None
        assert bench.recorded_traffic(key, "another_workload", sources) is None
        # a different source set hashes differently: the record no longer applies
        assert bench.recorded_traffic(key, wl, [os.path.join(ROOT, "bench.py")]) is None
    assert bench.recorded_traffic("no_such_kernel", "gmm16k_d64_fp32") is None


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
