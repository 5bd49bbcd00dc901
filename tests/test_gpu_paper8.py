"""The paper's own ingest on the GPU: 8-bit (and 16-bit) 2200-sample frames
through the mixed-radix (4, 5, 5, 11) FFT, against the FP64 oracle.

Bars: tooth amplitudes within 1e-4 relative of the oracle on comb teeth
(against the frame's RMS bin amplitude for arbitrary bins); centres within
1e-3 FWHM on >= 99.9 % of frames."""

import sys

import numpy as np
import pytest

import oracle
import synth
from oracle.fano import fano_fit_batch
from oracle.pipeline import process_batch_fano
from parity_util import MAG_RTOL, PASS_FRACTION, centre_parity, mag_rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12988_amd as cg  # noqa: E402
from test_gpu_fano import fano_parity  # noqa: E402

DEV = torch.device("cuda:0")
W, Q, DBAR, BBAR = 8.03, 4.0, 0.6, 1.0


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dtype", ["int8", "int16"])
@pytest.mark.parametrize("nf", [1, 5, 777])
def test_mixed_radix_teeth_match_oracle_on_random_frames(dtype, nf):
    """Random full-scale frames, 440 random bins including DC and Nyquist:
    amplitude error against the frame's RMS bin amplitude."""
    rng = np.random.default_rng(nf)
    lim = 128 if dtype == "int8" else 32768
    npd = np.int8 if dtype == "int8" else np.int16
    fr = rng.integers(-lim, lim, size=(nf, 2200)).astype(npd)
    bins = np.concatenate([[0, 1100], rng.choice(np.arange(1, 1100), 438, replace=False)])
    bins = bins.astype(np.int32)
    plan = cg.Plan(2200, 2.2e9, bins, np.ones(440), sample_type=dtype)
    mag, _ = plan.teeth(torch.from_numpy(fr).to(DEV), want_y=False)
    torch.cuda.synchronize()
    ora = oracle.tooth_magnitudes(fr, bins)
    rms = np.sqrt(np.mean(np.abs(np.fft.rfft(fr.astype(np.float64), axis=1)) ** 2, axis=1))
    err = np.abs(mag.cpu().numpy() - ora) / rms[:, None]
    _say(f"{dtype} nf={nf}: max error / rms bin amplitude {err.max():.2e}")
    assert err.max() <= MAG_RTOL


def test_paper_comb_teeth_and_centres_cold():
    """The paper's comb on 8-bit frames with the Lorentzian cold start: teeth
    within 1e-4 relative, centres at the bar."""
    spec = synth.StreamSpec(name="p8l", n=2200, fs=2.2e9, bins=synth.tooth_bins_paper_2200(),
                            width=(4.0, 16.0), depth=(0.6, 0.6), snr_db=(20.0, 50.0), bits=8,
                            sample_dtype="int8")
    bt = synth.make_batch(spec, 1500, seed=81)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    ora = oracle.process_batch(bt.frames, spec.bins, ref)
    plan = cg.Plan(2200, spec.fs, spec.bins, ref, sample_type="int8")
    out = plan.process(torch.from_numpy(bt.frames).to(DEV),
                       want=("params", "teeth", "iters", "status"))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    me = mag_rel_err(g["teeth"], ora["mags"]).max()
    res = centre_parity(ora["y"], g["params"], ora["params"], ora["status"], ora["chi2"])
    _say(f"  teeth max rel {me:.2e}; centres {res['fraction']:.5f} of {res['n']} "
         f"(exempt {res['exempt']}), iters gpu {g['iters'].mean():.2f} oracle "
         f"{ora['iters'].mean():.2f}")
    assert me <= MAG_RTOL
    assert res["fraction"] >= PASS_FRACTION, res
    assert abs(g["iters"].mean() - ora["iters"].mean()) < 0.5


def test_paper_configuration_fano_end_to_end():
    """The paper's whole configuration: 8-bit 2200-sample frames, its comb,
    its boxed Fano fit."""
    spec = synth.spec_paper8()
    bt = synth.make_batch(spec, 1500, seed=82)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    ora = process_batch_fano(bt.frames, spec.bins, ref, W, Q, DBAR, BBAR)
    plan = cg.Plan(2200, spec.fs, spec.bins, ref, sample_type="int8")
    plan.set_fano(W, Q, DBAR, BBAR)
    out = plan.process(torch.from_numpy(bt.frames).to(DEV), flags=cg.FIT_FANO,
                       want=("params", "teeth", "iters", "status"))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    assert mag_rel_err(g["teeth"], ora["mags"]).max() <= MAG_RTOL
    res = fano_parity(ora["y"], g["params"], ora["params"], ora["status"], ora["chi2"], W, Q)
    _say(f"  fano centres {res['fraction']:.5f} of {res['n']}, max {res['max_err']:.2e}; "
         f"iters gpu {g['iters'].mean():.2f} oracle {ora['iters'].mean():.2f}")
    assert res["fraction"] >= PASS_FRACTION, res
    assert abs(g["iters"].mean() - ora["iters"].mean()) < 0.5


def test_paper_configuration_full_batch_sampled():
    """65536 x 2200 int8 frames (the benchmark's batch), the Fano fit; 4096
    sampled frames fitted by the oracle from the whole batch's start points."""
    spec = synth.spec_paper8()
    nf = 65536
    bt = synth.make_batch(spec, nf, seed=83)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    plan = cg.Plan(2200, spec.fs, spec.bins, ref, sample_type="int8")
    plan.set_fano(W, Q, DBAR, BBAR)
    out = plan.process(torch.from_numpy(bt.frames).to(DEV), flags=cg.FIT_FANO,
                       want=("params", "iters", "status"))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    y = oracle.normalize(oracle.tooth_magnitudes(bt.frames, spec.bins), ref)
    p0 = oracle.initial_guess(y)
    rows = np.sort(np.random.default_rng(4).choice(nf, 4096, replace=False))
    p_or, it_or, st_or, c2_or = fano_fit_batch(y, p0[:, 0], W, Q, DBAR, BBAR, rows=rows)
    res = fano_parity(y[rows], g["params"][rows], p_or, st_or, c2_or, W, Q)
    _say(f"  full batch: {res['fraction']:.5f} of {res['n']}, iters gpu "
         f"{g['iters'][rows].mean():.2f} oracle {it_or.mean():.2f}")
    assert res["fraction"] >= PASS_FRACTION, res


def test_paper_geometry_errors_and_pipeline():
    bins = synth.tooth_bins_paper_2200()
    with pytest.raises(cg.CombGpuError):
        cg.Plan(2048, 2.2e9, bins[:100], np.ones(100), sample_type="int8")   # int8 needs 2200
    with pytest.raises(cg.CombGpuError):
        cg.Plan(2000, 2.2e9, bins[:100], np.ones(100))                       # not a supported length
    spec = synth.spec_paper8()
    bt = synth.make_batch(spec, 600, seed=84)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    plan = cg.Plan(2200, spec.fs, spec.bins, ref, sample_type="int8")
    fr = torch.from_numpy(bt.frames).to(DEV)
    with pytest.raises(cg.CombGpuError):
        plan.process(fr, flags=cg.DFT_MFMA_BF16X3)
    with pytest.raises(TypeError):
        plan.process(fr.to(torch.int16))                                    # wrong sample type
    # the host-ring pipeline carries 8-bit bursts (half the bytes of int16)
    plan.set_fano(W, Q, DBAR, BBAR)
    pipe = cg.Pipeline([plan], [cg.FIT_FANO], slots_per_stream=3, max_burst_frames=300,
                       keep_results=True, lanes=2, host_ring=True)
    pipe.put(0, np.ascontiguousarray(bt.frames[:300]), 0)
    pipe.put(0, np.ascontiguousarray(bt.frames[300:600]), 1)
    pipe.drain(60000)
    st = pipe.stats()
    assert st["bytes"] == 600 * 2200
    for j in range(2):
        got = pipe.read(0)
        want = plan.process(fr[300 * j:300 * (j + 1)].contiguous(), flags=cg.FIT_FANO,
                            want=("params",))["params"].cpu().numpy()
        assert got[0] == j and np.array_equal(got[1], want)
    pipe.close()
