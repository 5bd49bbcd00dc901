"""Degenerate batch sizes through every fit form: empty batches, single
frames and batches shorter than the 7x7 median window (the window then
replicates the batch's edge frames on both sides), against the FP64 oracle
on the same frames."""

import os
import sys

import numpy as np
import pytest

import oracle
import oracle.pipeline
import synth
from parity_util import MAG_RTOL, PASS_FRACTION, centre_parity, mag_rel_err, warm_compared

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12988_amd as cg  # noqa: E402
from test_gpu_fano import fano_parity  # noqa: E402

DEV = torch.device("cuda:0")
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2307_12988_amd", "data", "warmstart_learned.npz")
W, Q, DBAR, BBAR = 8.03, 4.0, 0.6, 1.0


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nf", [1, 2, 3, 6, 7, 8])
def test_short_batches_cold_path(nf):
    """Fewer frames than (or as many as) the median window: amplitudes, start
    points (bit-identical on the same spectra) and centres."""
    spec = synth.spec_tiny()
    bt = synth.make_batch(spec, nf, seed=40 + nf)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    ora = oracle.process_batch(bt.frames, spec.bins, ref)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, ref)
    out = plan.process(torch.from_numpy(bt.frames).to(DEV),
                       want=("params", "status", "teeth", "y"))
    torch.cuda.synchronize()
    assert mag_rel_err(out["teeth"].cpu().numpy(), ora["mags"]).max() <= MAG_RTOL
    y = out["y"]
    p0_gpu, med = plan.init_spectra(y, want_median=True)
    torch.cuda.synchronize()
    y_np = y.cpu().numpy()
    assert np.array_equal(med.cpu().numpy(), oracle.median7x7(y_np))
    assert np.array_equal(p0_gpu.cpu().numpy(), oracle.initial_guess(y_np))
    res = centre_parity(ora["y"], out["params"].cpu().numpy(), ora["params"], ora["status"],
                        ora["chi2"])
    _say(f"nf={nf}: centres {res['fraction']:.3f} of {res['n']}, max {res['max_err']:.2e}")
    assert res["fraction"] >= PASS_FRACTION, res


@pytest.mark.parametrize("nf", [0, 1, 3, 5])
def test_short_batches_paper_configuration(nf):
    """The paper's 8-bit 2200-sample frames with the boxed Fano fit."""
    spec = synth.spec_paper8()
    bt = synth.make_batch(spec, max(nf, 1), seed=60 + nf)
    frames = bt.frames[:nf]
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, ref, sample_type="int8")
    plan.set_fano(W, Q, DBAR, BBAR)
    out = plan.process(torch.from_numpy(np.ascontiguousarray(frames)).to(DEV),
                       flags=cg.FIT_FANO, want=("params", "status", "teeth"))
    torch.cuda.synchronize()
    assert out["params"].shape == (nf, 4)
    if nf == 0:
        return
    ora = oracle.pipeline.process_batch_fano(frames, spec.bins, ref, W, Q, DBAR, BBAR)
    assert mag_rel_err(out["teeth"].cpu().numpy(), ora["mags"]).max() <= MAG_RTOL
    res = fano_parity(ora["y"], out["params"].cpu().numpy(), ora["params"], ora["status"],
                      ora["chi2"], W, Q)
    _say(f"paper8 nf={nf}: centres {res['fraction']:.3f} of {res['n']}")
    assert res["fraction"] >= PASS_FRACTION, res


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not built")
@pytest.mark.parametrize("nf", [0, 1, 4])
def test_short_batches_warm_path(nf):
    """The learned warm start (network, polish, fallback, refit) on tiny
    batches."""
    d = np.load(WEIGHTS)
    spec = synth.spec_learned()
    bt = synth.make_batch(spec, max(nf, 1), seed=80 + nf)
    frames = np.ascontiguousarray(bt.frames[:nf])
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, ref)
    plan.set_mlp(d["params"], d["out_mean"], d["out_std"], float(d["noise_floor"]))
    out = plan.process(torch.from_numpy(frames).to(DEV), flags=cg.FIT_WARM_MLP,
                       want=("params", "status"))
    torch.cuda.synchronize()
    assert out["params"].shape == (nf, 4)
    if nf == 0:
        return
    ora = oracle.pipeline.process_batch_warm(frames, spec.bins, ref,
                                             d["params"].astype(np.float64), d["out_mean"],
                                             d["out_std"], float(d["noise_floor"]))
    assert np.array_equal(out["status"].cpu().numpy() == 3, ora["status"] == 3)
    res = centre_parity(ora["y"], out["params"].cpu().numpy(), ora["params"],
                        warm_compared(ora["status"]), ora["chi2"])
    _say(f"warm nf={nf}: centres {res['fraction']:.3f} of {res['n']}")
    assert res["fraction"] >= PASS_FRACTION, res


@pytest.mark.parametrize("flag", [cg.DFT_MFMA_BF16X3, cg.DFT_MFMA_FP16X2, cg.DFT_MFMA_FP16])
@pytest.mark.parametrize("nf", [0, 1, 17])
def test_short_batches_matrix_core_forms(flag, nf):
    """The matrix-core tooth transforms on batches smaller than one tile of
    frames (an empty batch writes nothing)."""
    spec = synth.spec_precision()
    bt = synth.make_batch(spec, max(nf, 1), seed=90 + nf)
    frames = np.ascontiguousarray(bt.frames[:nf])
    plan = cg.Plan(spec.n, spec.fs, spec.bins, np.ones(spec.k, np.float32))
    mag, _ = plan.teeth(torch.from_numpy(frames).to(DEV), flags=flag, want_y=False)
    torch.cuda.synchronize()
    assert mag.shape == (nf, spec.k)
    if nf == 0:
        return
    bar = {cg.DFT_MFMA_BF16X3: 1e-4, cg.DFT_MFMA_FP16X2: 1e-3, cg.DFT_MFMA_FP16: 3e-3}[flag]
    err = mag_rel_err(mag.cpu().numpy(), oracle.tooth_magnitudes(frames, spec.bins))
    assert err.max() <= bar


@pytest.mark.parametrize("k", [1, 2, 3])
def test_fewer_teeth_than_parameters(k):
    """One to three teeth for a four-parameter dip.  One tooth: the damped
    normal matrix has a zero column (no tooth sees the width or the centre
    move), and both sides report every fit singular.  Two or three teeth: the
    dip can pass through every tooth, so fits are not unique and their
    iteration counts depend on rounding; only the outcome is checked: a
    valid status, and a final chi2 no larger than at the start point."""
    spec = synth.StreamSpec(name="few", n=512, fs=1e9, bins=np.arange(10, 10 + 5 * k, 5),
                            width=(4, 16), snr_db=(30, 50))
    bt = synth.make_batch(spec, 40, seed=k)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    ora = oracle.process_batch(bt.frames, spec.bins, ref)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, ref)
    out = plan.process(torch.from_numpy(bt.frames).to(DEV), want=("params", "status", "y"))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    if k == 1:
        assert np.all(st == cg.FIT_SINGULAR) and np.all(ora["status"] == 2)
        return
    assert np.all(np.isin(st, (0, 1, 2)))
    y = out["y"].cpu().numpy().astype(np.float64)
    p = out["params"].cpu().numpy()
    p0 = oracle.initial_guess(out["y"].cpu().numpy())
    for f in np.nonzero(st != 2)[0]:
        assert oracle.chi2_at(y[f], p[f]) <= oracle.chi2_at(y[f], p0[f]) * (1 + 1e-5) + 1e-12


@pytest.mark.parametrize("k,nf", [(220, 1000), (100, 37), (440, 70), (7, 20)])
def test_start_centres_equal_full_start_points(k, nf):
    """cg_start_centres writes the centre cg_init_spectra writes (column 0)
    and leaves the other columns alone."""
    rng = np.random.default_rng(k + nf)
    y = (1.0 - 0.5 * rng.random((nf, k))).astype(np.float32)
    plan = cg.Plan(2048, 1e9, np.arange(1, k + 1), np.ones(k))
    yt = torch.from_numpy(y).to(DEV)
    p0, _ = plan.init_spectra(yt)
    c = torch.full((nf, 4), -3.0, dtype=torch.float32, device=DEV)
    plan.start_centres(yt, out_p0=c)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    assert np.array_equal(c[:, 0], p0.cpu().numpy()[:, 0])
    assert np.all(c[:, 1:] == -3.0)
    assert np.array_equal(c[:, 0], oracle.initial_guess(y)[:, 0])
