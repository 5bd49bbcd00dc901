"""Precision form: tooth DFT on the matrix cores, per form, against the FP64
oracle.  Bars, each derived from the form's rounding:
  BF16X3   samples split exactly, basis carried to ~2^-17: max rel amplitude
           error <= 1e-4 (the same bar as the FFT path);
  FP16X2   samples split exactly, basis rounded to fp16 (rel 2^-12 per entry):
           rms rel error <= 1e-4, max <= 1e-3;
  FP16     samples and basis rounded to fp16: rms <= 3e-4, max <= 3e-3.
Centres through the whole path must meet the 1e-3 FWHM bar for every form."""

import sys

import numpy as np
import pytest

import oracle
import synth
from parity_util import MAG_RTOL, PASS_FRACTION, centre_parity, mag_rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12988_amd as cg  # noqa: E402

DEV = torch.device("cuda:0")
FORMS = {"bf16x3": (cg.DFT_MFMA_BF16X3, 1e-4, 1e-4), "fp16x2": (cg.DFT_MFMA_FP16X2, 1e-3, 1e-4),
         "fp16": (cg.DFT_MFMA_FP16, 3e-3, 3e-4)}


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("n,k,nf", [(4096, 220, 500), (2048, 220, 333), (512, 100, 70),
                                    (8192, 440, 65), (1024, 37, 129)])
def test_mfma_amplitudes(form, n, k, nf):
    flag, max_bar, rms_bar = FORMS[form]
    spec = synth.StreamSpec(name="p", n=n, fs=1.1e9, bins=synth.tooth_bins_interleaved(n, k),
                            width=(4, 16), snr_db=(20, 50))
    bt = synth.make_batch(spec, nf, seed=n + k + 2)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    plan = cg.Plan(n, spec.fs, spec.bins, ref)
    mag, y = plan.teeth(torch.from_numpy(bt.frames).to(DEV), flags=flag)
    torch.cuda.synchronize()
    m_or = oracle.tooth_magnitudes(bt.frames, spec.bins)
    err = mag_rel_err(mag.cpu().numpy(), m_or)
    _say(f"{form} n={n} k={k}: max {err.max():.2e} rms {np.sqrt(np.mean(err ** 2)):.2e}")
    assert err.max() <= max_bar
    assert np.sqrt(np.mean(err ** 2)) <= rms_bar
    assert mag_rel_err(y.cpu().numpy(), oracle.normalize(m_or, ref)).max() <= max_bar * 1.01


@pytest.mark.parametrize("form", list(FORMS))
def test_mfma_whole_path_centres(form):
    flag = FORMS[form][0]
    spec = synth.spec_precision()
    bt = synth.make_batch(spec, 2048, seed=2)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    ora = oracle.process_batch(bt.frames, spec.bins, ref)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, ref)
    out = plan.process(torch.from_numpy(bt.frames).to(DEV), flags=flag,
                       want=("params", "status"))
    torch.cuda.synchronize()
    res = centre_parity(ora["y"], out["params"].cpu().numpy(), ora["params"], ora["status"],
                        ora["chi2"])
    _say(f"{form}: centre fraction {res['fraction']:.5f} max_err {res['max_err']:.2e}")
    assert res["fraction"] >= PASS_FRACTION, res


def test_precision_full_size_sampled():
    """The precision workload at its full size and launch shape (131072 frames
    x 4096 int16, 220 teeth, one launch per form): every 61st frame and the
    last one against the FP64 oracle, at each form's bars (the FFT at 1e-4)."""
    spec = synth.spec_precision()
    bt = synth.make_batch(spec, 16384, seed=2)
    frames = np.tile(bt.frames, (8, 1))                 # 131072 frames
    nf = frames.shape[0]
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, ref)
    sample = np.unique(np.concatenate([np.arange(0, nf, 61), [nf - 1]]))
    m_or = oracle.tooth_magnitudes(frames[sample], spec.bins)
    fr = torch.from_numpy(frames).to(DEV)
    forms = {"fft": (cg.DFT_FFT, MAG_RTOL, MAG_RTOL)}
    forms.update(FORMS)
    for name, (flag, max_bar, rms_bar) in forms.items():
        _say(f"precision full size: {name}")
        mag, _ = plan.teeth(fr, flags=flag, want_y=False)
        torch.cuda.synchronize()
        err = mag_rel_err(mag[torch.from_numpy(sample).to(DEV)].cpu().numpy(), m_or)
        _say(f"  {len(sample)} sampled frames: max {err.max():.2e} rms "
             f"{np.sqrt(np.mean(err ** 2)):.2e}")
        assert err.max() <= max_bar
        assert np.sqrt(np.mean(err ** 2)) <= rms_bar
        del mag
    plan.close()


def test_mfma_rejects_misaligned_frames():
    spec = synth.spec_tiny()
    plan = cg.Plan(spec.n, spec.fs, spec.bins, np.ones(spec.k))
    buf = torch.zeros(4 * spec.n + 8, dtype=torch.int16, device=DEV)
    fr = buf[2:2 + 4 * spec.n].view(4, spec.n)        # 4-byte but not 16-byte aligned
    with pytest.raises(cg.CombGpuError):
        plan.teeth(fr, flags=cg.DFT_MFMA_BF16X3)
    mag, _ = plan.teeth(fr, flags=cg.DFT_FFT)         # the FFT path accepts it
    torch.cuda.synchronize()
