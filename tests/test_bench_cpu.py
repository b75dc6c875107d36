"""Host-side checks of bench.py: the one-GPU guard, the oracle baseline record
and the source hash that gates the profiled traffic figure."""
import json
import os
import subprocess
import sys

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]


def test_cpu_baseline_record_on_a_small_uneven_batch():
    w = W.uneven_mixed(n_worlds=32, steps=3)
    rec = bench.cpu_baseline(w, seconds=0.5)
    assert rec["kind"] == "oracle" and rec["unit"] == "drone-steps/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    # the sample is every 16th world: worlds 0 and 16 of 32
    n = int(np.diff(w.world_offsets())[[0, 16]].sum())
    assert f"(2 worlds, {n} drones)" in rec["sample"]


def test_source_hash_is_a_stable_sha256():
    a, b = bench.kernel_sources_sha256(), bench.kernel_sources_sha256()
    assert a == b and len(a) == 64
    int(a, 16)
    # empty until the current kernels have been profiled
    assert len(bench.PROFILED_TRAFFIC["sources_sha256"]) in (0, 64)


def test_one_thread_cpu_baseline_uses_one_thread():
    import torch
    before = torch.get_num_threads()
    w = W.uneven_mixed(n_worlds=256, steps=2)
    rec = bench.cpu_baseline(w, seconds=0.3, threads=1)
    assert rec["cores"] == 1 and rec["value"] > 0
    assert "(2 worlds," in rec["sample"]          # every 128th world
    assert torch.get_num_threads() == before
