"""Host-side helpers of bench.py: the seeded batch generator and the pool
builder every workload uses (no device needed), the traffic table's source
hashes, and the refusal of more than one GPU."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def test_generator_returns_frames_reference_and_truth():
    spec = synth.spec_tiny()
    b, frames, ref, (centre, width) = bench._gen((spec, 16, 5, 1))
    assert b == 1
    assert frames.shape == (16, spec.n) and frames.dtype == np.int16
    assert ref.shape[1] == spec.n and ref.dtype == np.int16
    assert centre.shape == (16,) and width.shape == (16,) and np.all(width > 0)
    again = synth.make_batch(spec, 16, seed=5, batch_index=1)
    assert np.array_equal(frames, again.frames) and np.array_equal(centre, again.centre)


def test_pool_with_and_without_truth():
    spec = synth.spec_tiny()
    frames, ref = bench.make_pool(spec, 8, 2, workers=1)
    assert len(frames) == 2 and frames[0].shape == (8, spec.n)
    frames2, ref2, truths = bench.make_pool(spec, 8, 2, workers=1, truth=True)
    assert all(np.array_equal(a, b) for a, b in zip(frames, frames2))
    assert len(truths) == 2 and truths[1][0].shape == (8,)


def test_traffic_entries_name_existing_sources():
    for kernel, (sources, digest, rd, wr) in bench.TRAFFIC.items():
        for name in sources:
            assert os.path.exists(os.path.join(ROOT, "paper_2307_12988_amd", "csrc", name)), name
        assert len(digest) == 16 and rd > 0 and wr > 0
        # the bytes while the sources still hash to the recorded digest, else null
        assert bench.traffic_bytes(kernel) in (rd + wr, None), kernel


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert res.returncode != 0
    assert "one GPU" in (res.stdout + res.stderr) or "1 GPU" in (res.stdout + res.stderr)
