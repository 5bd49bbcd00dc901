"""End-to-end checks of the oracle against the generator's ground truth."""

import numpy as np

import oracle
import synth


def test_noiseless_frames_recover_truth():
    """Without noise only the 14-bit quantisation perturbs the spectra, so the
    fitted dip matches the synthesis parameters to a small fraction of a tooth."""
    spec = synth.spec_tiny()
    bt = synth.make_batch(spec, 64, seed=5, noise=False)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins)
    out = oracle.process_batch(bt.frames, spec.bins, ref)
    assert np.all(out["status"] == 0)
    assert np.max(np.abs(out["params"][:, 0] - bt.centre)) < 2e-3 * 8
    assert np.max(np.abs(out["params"][:, 1] - bt.width)) < 1e-2
    assert np.max(np.abs(out["params"][:, 2] - bt.depth)) < 1e-3


def test_tiny_workload_centre_error_at_noise_limit():
    """At 40 dB SNR the centre error is the Cramer-Rao level of the tiny
    workload (about 1.4e-3 FWHM), and fits take a handful of iterations."""
    spec = synth.spec_tiny()
    bt = synth.make_batch(spec, 512, seed=0)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins)
    out = oracle.process_batch(bt.frames, spec.bins, ref)
    assert np.all(out["status"] == 0)
    err = (out["params"][:, 0] - bt.centre) / bt.width
    rms = np.sqrt(np.mean(err ** 2))
    assert 0.7e-3 < rms < 2.5e-3
    assert 3 <= np.median(out["iters"]) <= 6
