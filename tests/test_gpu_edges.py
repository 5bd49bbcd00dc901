"""Degenerate batch sizes through every fit form: empty batches, single
frames and batches shorter than the 7x7 median window (the window then
replicates the batch's edge frames on both sides), against the FP64 oracle
on the same frames."""

import os
import sys
import zlib

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


def _dip_rows(nf, k, rng, centre, depth=0.6, width=8.0, noise=0.02, step=None):
    """Lorentzian dips at the given centres (one per frame) plus Gaussian
    noise, optionally rounded to multiples of `step` (many equal values)."""
    x = np.arange(k)
    y = 1.0 - depth / (1.0 + (2.0 * (x[None, :] - centre[:, None]) / width) ** 2)
    y = y + noise * rng.standard_normal((nf, k))
    if step:
        y = np.round(y / step) * step
    return y.astype(np.float32)


def _centre_case(case, k, nf, rng):
    t = np.arange(nf)
    mid = (k - 1) / 2
    if case == "dip":            # the stream's motion: +-10 teeth at 1/42 of the frame rate
        return _dip_rows(nf, k, rng, mid + min(10.0, k / 4) * np.sin(2 * np.pi * t / 42.0))
    if case == "dip_low_edge":   # minima on and next to the first tooth
        return _dip_rows(nf, k, rng, 1.5 + 1.5 * np.sin(2 * np.pi * t / 13.0))
    if case == "dip_high_edge":
        return _dip_rows(nf, k, rng, k - 2.5 + 1.5 * np.sin(2 * np.pi * t / 13.0))
    if case == "noisy":          # the bounds overlap widely: most columns are filtered
        return _dip_rows(nf, k, rng, mid + 0 * t, depth=0.05, noise=0.05)
    if case == "quantised":      # equal values everywhere, bounds equal to u
        return _dip_rows(nf, k, rng, mid + 6.0 * np.sin(2 * np.pi * t / 29.0), noise=0.05,
                         step=1 / 16)
    if case == "two_equal_dips":  # two identical minima per row: the first one counts
        prof = 1.0 - 0.6 / (1.0 + (2.0 * (np.arange(k) - k // 4) / 6.0) ** 2)
        row = np.minimum(prof, prof[::-1]).astype(np.float32)
        return np.repeat(row[None, :], nf, axis=0)
    if case == "flat":
        return np.ones((nf, k), np.float32)
    raise ValueError(case)


@pytest.mark.parametrize("case,k,nf", [
    ("dip", 220, 2000), ("dip", 100, 333), ("dip", 440, 300), ("dip", 7, 50),
    ("dip_low_edge", 220, 500), ("dip_high_edge", 220, 500), ("dip_high_edge", 61, 100),
    ("noisy", 220, 500), ("quantised", 220, 1000), ("quantised", 33, 77),
    ("two_equal_dips", 220, 64), ("two_equal_dips", 40, 17), ("flat", 220, 40), ("flat", 1, 5)])
def test_start_centres_pruned_filter_cases(case, k, nf):
    """The centre-only kernel filters exactly only the columns whose window
    bounds (the smallest and largest median of the window's seven row
    segments) leave room for a row's minimum.  These cases put the minimum on
    the edge teeth, tie it between columns, make values equal to the bounds
    and flatten the rows, so that the bounds keep few, many or all columns;
    every centre must be the oracle's (first index of the filtered row's
    minimum) and the full start-point kernel's."""
    rng = np.random.default_rng(zlib.crc32(f"{case} {k} {nf}".encode()))
    y = _centre_case(case, k, nf, rng)
    plan = cg.Plan(2048, 1e9, np.arange(1, k + 1), np.ones(k))
    yt = torch.from_numpy(y).to(DEV)
    c = torch.full((nf, 4), -3.0, dtype=torch.float32, device=DEV)
    plan.start_centres(yt, out_p0=c)
    p0, _ = plan.init_spectra(yt)
    torch.cuda.synchronize()
    got = c.cpu().numpy()[:, 0]
    want = oracle.initial_guess(y)[:, 0]
    bad = np.nonzero(got != want)[0]
    _say(f"{case} k={k} nf={nf}: {len(bad)} centres differ from the oracle"
         + (f", first frame {bad[0]}: {got[bad[0]]} vs {want[bad[0]]}" if len(bad) else ""))
    assert len(bad) == 0
    assert np.array_equal(got, p0.cpu().numpy()[:, 0])
    if case == "two_equal_dips":
        # the filtered row is flat at its minimum over five teeth in each
        # dip: the first of those ten equal values counts
        assert np.all(got == k // 4 - 2)


def test_start_centres_on_the_fano_stream():
    """Start centres of the Fano stream's spectra (the GPU path's own y) equal
    the oracle's on the same spectra."""
    spec = synth.spec_fano()
    bt = synth.make_batch(spec, 1500, seed=77)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, np.ones(spec.k, dtype=np.float32))
    ref = plan.reference_from_frames(torch.from_numpy(bt.ref_frames).to(DEV)).cpu().numpy()
    plan.set_reference(ref)
    _, y = plan.teeth(torch.from_numpy(bt.frames).to(DEV), want_mag=False, want_y=True)
    c = torch.zeros((1500, 4), dtype=torch.float32, device=DEV)
    plan.start_centres(y, out_p0=c)
    torch.cuda.synchronize()
    got = c.cpu().numpy()[:, 0]
    want = oracle.initial_guess(y.cpu().numpy())[:, 0]
    _say(f"Fano stream: {np.sum(got != want)} of 1500 centres differ")
    assert np.array_equal(got, want)


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
