"""bench.py's command-line contract and the counter records it reports (no GPU):
a run on more than one GPU is refused with a message before anything touches a
GPU, and the HBM traffic records of the headline kernel and of the recorded
score replay were taken from the kernel sources as they stand (bench.py
reports a record only while its sources hash to the recorded SHA-1)."""
import importlib.util
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("gpus", [2, 8])
def test_more_than_one_gpu_is_refused(gpus):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(gpus)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("kernel", ["hop_wave", "replay_logged"])
def test_traffic_record_matches_the_kernel_sources(kernel):
    b = _bench()
    rec = b.measured_traffic(kernel)
    assert rec is not None, f"profiles/{b.TRAFFIC[kernel][0]} was taken from other sources"
    # the record's total is its two scaled counters (KiB per launch)
    total = (rec["fetch_kib_per_launch"] * rec["fetch_scale"] + rec["write_kib_per_launch"] * rec["write_scale"]) * 1024
    assert abs(total - rec["hbm_bytes_per_launch"]) <= 1e-3 * total


def test_every_traffic_record_parses():
    b = _bench()
    for kernel, (md, src) in b.TRAFFIC.items():
        text = open(os.path.join(ROOT, "profiles", md)).read()
        m = re.search(r"```json\n(.*?)\n```", text, re.S)
        assert m, md
        rec = json.loads(m.group(1))
        assert rec["kernel"].startswith(kernel) and len(rec["kernel_sha1"]) == 40
        assert os.path.exists(os.path.join(ROOT, "paper_2511_09413_amd", "csrc", src))
