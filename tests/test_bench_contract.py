"""The benchmark's contract, checked on the CPU: one GPU only, a loud exit
without a GPU, the algorithmic byte counts it divides by, and the threaded
oracle leg (raw-slice shards) on a small cover."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_no_gpu_exits_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = _run("--steps", "1", "--warmup", "0")
    assert r.returncode != 0 and "needs a GPU" in r.stderr
    assert not r.stdout.strip(), "no JSON line without a measurement"


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
def test_algorithmic_bytes(k):
    """Embed moves the cover in and the stego out plus the stream (2n + |S|);
    extract reads the F = ceil(8|S| / k) carrying bytes and writes the
    message.  At full capacity of the 8192x8192x3 cover, F = n exactly for
    k dividing 8."""
    n = 8192 * 8192 * 3
    ln = oracle.capacity(n, k)
    s = 4 + ln
    assert bench.embed_bytes(n, ln) == 2 * n + s
    f = -(-8 * s // k)
    assert bench.extract_bytes(n, ln, k) == f + ln
    if 8 % k == 0:
        assert f == n


def test_threaded_oracle_leg():
    """The threaded CPU baseline cuts the cover into shards at multiples of 8
    bytes and runs each as a raw slice: its decoded stream checks out at
    every k of the workload, and the figure is a rate over the same bytes."""
    n = 3 * 65536 + 8 * 37
    cover = np.random.default_rng(7).integers(0, 256, n, dtype=np.uint8)
    msgs = {k: np.random.default_rng(10 + k).integers(0, 256, oracle.capacity(n, k), dtype=np.uint8)
            for k in bench.KS}
    r = bench.cpu_baseline_threads(cover, msgs, 5, min_seconds=0.0)
    assert r["kind"] == "oracle" and r["cores"] == 5 and r["value"] > 0 and r["unit"] == "GB/s"
    assert r["sample"].startswith("1 full step ")
    many = bench.cpu_baseline_threads(cover, msgs, 3, min_seconds=1e9, max_steps=2)
    assert many["sample"].startswith("2 full steps ") and many["cores"] == 3


def test_host_cpus_reported():
    """The baseline states the host's CPU count, the cores this process may
    use and the share the threaded oracle takes (at most 16)."""
    h = bench.host_cpus()
    assert h["os_cpu_count"] == os.cpu_count()
    assert 1 <= h["cpu_share"] <= min(16, h["affinity_cpus"])
    assert h["cpu_model"] is None or "family" in h["cpu_model"]


def test_single_thread_oracle_leg_repeats_to_its_time_floor():
    """The single-thread baseline repeats whole steps until its time floor
    (at least one step, at most max_steps) and counts the bytes of each."""
    import numpy as np

    import oracle

    cover = (np.arange(4096, dtype=np.uint32) * 37 % 251).astype(np.uint8)
    msgs = {k: np.full(oracle.capacity(cover.size, k), 0x5A, np.uint8) for k in bench.KS}
    one = bench.cpu_baseline(cover, msgs, min_seconds=0.0)
    assert one["sample"].startswith("1 full step:") and one["cores"] == 1
    many = bench.cpu_baseline(cover, msgs, min_seconds=1e9, max_steps=3)
    assert many["sample"].startswith("3 full steps:")
    assert one["value"] > 0 and many["value"] > 0


def test_batched_traffic_entries_are_current():
    """While the committed counter profile of the batched kernels matches
    their sources, the bench reads a traffic figure per batched launch, the
    clip's within 1 % of its algorithmic bytes."""
    alg = {"clip_frames_embed": 7698240000, "clip_frames_extract": 2099519996}
    if bench.stored_batch_traffic("batched_embed") is None:
        pytest.skip("batched kernel sources changed since the counters were taken: retake them")
    for launch in ("batched_embed", "batched_extract", "clip_frames_embed", "clip_frames_extract"):
        t = bench.stored_batch_traffic(launch)
        assert isinstance(t, int) and t > 0, launch
        if launch in alg:
            assert abs(t / alg[launch] - 1) < 0.01, launch
    r = bench.batched_roofline(8e9, 2e-3, "batched_embed", "stream events")
    assert r["achieved"] == 4000.0 and r["frac"] == 0.5 and r["bound"] == "hbm"
