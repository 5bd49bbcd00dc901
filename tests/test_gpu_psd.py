"""Displacement PSD and mechanical resonance fit on the GPU against the FP64
oracle.

Bars.  PSD: relative error per band bin <= 1e-3.  The FP32 transforms carry
an absolute error of about 2^-24 sqrt(log2 L) of the segment's largest bin
amplitude into every bin; the band's power spans up to about 10^4 between the
resonance and the floor, i.e. 10^2 in amplitude, so a floor bin's power can
move by 2 * 10^2 * 2^-24 * 4 ~ 5e-5 relative, and 1e-3 leaves room for
the sums.  Fit: f0 within 1e-3 of the resonance linewidth f0/Q and Q within
1e-3 relative of the oracle's fit of the oracle's PSD."""

import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import psd as opsd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12988_amd as cg  # noqa: E402

DEV = torch.device("cuda:0")
FS, F0, Q = 1.0e6, 23.7e3, 115.0
PSD_RTOL = 1e-5


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("seg,n", [(16384, 1 << 18), (65536, 1 << 20), (32768, 100001),
                                   (131072, 1 << 19)])
def test_psd_matches_oracle(seg, n):
    x = synth.make_displacement(n, FS, F0, Q, drive=1e-3, floor=2e-3, drift=1e-6, seed=seg)
    x = x + np.float32(110.0)                       # centres sit around the comb's middle
    k_lo, nb = cg.psd_band(seg, FS, 15e3, 35e3)
    got = cg.psd_welch(torch.from_numpy(x).to(DEV), FS, seg, k_lo, nb).cpu().numpy()
    want = opsd.welch_band(x.astype(np.float64), FS, seg, k_lo, nb)
    rel = np.abs(got - want) / want
    _say(f"seg={seg} n={n}: {nb} bins, max rel {rel.max():.2e}, median {np.median(rel):.2e}")
    # FP32 FFT of 2^13..2^16 complex points: about eps * sqrt(passes) of the
    # segment's RMS bin per bin; the band's bins sit within a few decades of
    # that RMS, and the FP64 sums over segments add nothing (measured <= 9e-7)
    assert rel.max() <= PSD_RTOL


def test_psd_band_edges_and_errors():
    x = synth.make_displacement(1 << 16, FS, F0, Q, 1e-3, 1e-3, 0.0, seed=3)
    xt = torch.from_numpy(x).to(DEV)
    # DC and Nyquist bins of a 16384 segment
    for k_lo, nb in ((0, 5), (8192 - 4, 5)):
        got = cg.psd_welch(xt, FS, 16384, k_lo, nb).cpu().numpy()
        want = opsd.welch_band(x.astype(np.float64), FS, 16384, k_lo, nb)
        rel = np.max(np.abs(got - want) / want)
        _say(f"bins {k_lo}..{k_lo + nb - 1}: max rel {rel:.2e}")
        # a bin's FP32 rounding scales with the segment's RMS bin, not with
        # the bin: relative error about 2 eps sqrt(passes) sqrt(P_mean / P_k);
        # near Nyquist this series has only its white floor, a few decades
        # below the mean power (measured 2.8e-5 there, 1.3e-6 at DC)
        assert rel <= 1e-4
    with pytest.raises(cg.CombGpuError):
        cg.psd_welch(xt[:1000].contiguous(), FS, 16384, 10, 10)       # shorter than a segment
    with pytest.raises(cg.CombGpuError):
        cg.psd_welch(xt, FS, 4096, 10, 10)                           # unsupported length
    with pytest.raises(cg.CombGpuError):
        cg.psd_welch(xt, FS, 16384, 8190, 10)                        # band past Nyquist


def test_resonance_fit_matches_oracle():
    x = synth.make_displacement(1 << 21, FS, F0, Q, drive=1e-3, floor=1e-2, drift=1e-6, seed=5)
    seg = 1 << 16
    k_lo, nb = cg.psd_band(seg, FS, 15e3, 35e3)
    g_psd = cg.psd_welch(torch.from_numpy(x).to(DEV), FS, seg, k_lo, nb)
    df = FS / seg
    out = cg.resonance_fit(g_psd, k_lo * df, df).cpu().numpy()
    o_psd = opsd.welch_band(x.astype(np.float64), FS, seg, k_lo, nb)
    f = (k_lo + np.arange(nb)) * df
    p, it, st, chi2 = opsd.oscillator_fit(f, o_psd)
    _say(f"gpu f0 {out[1]:.3f} Q {out[2]:.3f} it {out[5]:.0f} st {out[6]:.0f}; "
         f"oracle f0 {p[1]:.3f} Q {p[2]:.3f} it {it} st {st}")
    assert out[6] == 0 and st == 0
    assert abs(out[1] - p[1]) <= 1e-3 * p[1] / p[2]
    assert abs(out[2] / p[2] - 1) <= 1e-3
    # the same fit on the same (GPU) PSD agrees to rounding
    p2, _, _, _ = opsd.oscillator_fit(f, g_psd.cpu().numpy())
    assert abs(out[1] - p2[1]) <= 1e-6 * p2[1] / p2[2] and abs(out[2] / p2[2] - 1) <= 1e-6


def test_resonance_fit_exact_on_model_spectrum():
    f_first, df, nb = 15e3, 15.0, 1300
    f = f_first + df * np.arange(nb)
    truth = np.array([np.log(3e5), 23.7e3, 115.0, np.log(2e-9)])
    s = torch.from_numpy(opsd.oscillator(f, truth)).to(DEV)
    out = cg.resonance_fit(s, f_first, df).cpu().numpy()
    assert out[6] == 0
    assert np.allclose(out[:4], truth, rtol=1e-7, atol=1e-7), (out[:4], truth)
    with pytest.raises(cg.CombGpuError):
        cg.resonance_fit(s[:4].contiguous(), f_first, df)


def test_resonance_from_fitted_centres():
    """The whole chain: frames whose dip centre follows a displacement series
    with a resonance, the GPU path's fitted centres, their PSD and the fit.
    The recovered frequency is the series' own; the oracle gives the same f0
    and Q from the same centres."""
    spec = synth.spec_tiny()                       # 1024-sample frames at 1.024 GS/s
    fs_frame = spec.fs / spec.n                    # 1 MHz frame rate
    nfr = 1 << 18
    disp = synth.make_displacement(nfr, fs_frame, F0, Q, drive=2e-2, floor=0.0, drift=0.0,
                                   seed=9)
    bt = synth.make_batch(spec, nfr, seed=9, centre=spec.mid + disp)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, ref)
    cen = plan.process(torch.from_numpy(bt.frames).to(DEV))["params"][:, 0].contiguous()
    seg = 16384
    k_lo, nb = cg.psd_band(seg, fs_frame, 12e3, 40e3)
    g_psd = cg.psd_welch(cen, fs_frame, seg, k_lo, nb)
    df = fs_frame / seg
    out = cg.resonance_fit(g_psd, k_lo * df, df).cpu().numpy()
    f = (k_lo + np.arange(nb)) * df
    p, _, st, _ = opsd.oscillator_fit(f, opsd.welch_band(cen.cpu().numpy().astype(np.float64),
                                                         fs_frame, seg, k_lo, nb))
    _say(f"centres -> PSD -> fit: gpu f0 {out[1]:.1f} Hz Q {out[2]:.1f}; oracle f0 {p[1]:.1f} "
         f"Q {p[2]:.1f}; generator f0 {F0:.1f} Q {Q:.1f}")
    assert out[6] == 0 and st == 0
    assert abs(out[1] / F0 - 1) < 0.01
    assert abs(out[1] - p[1]) <= 1e-3 * p[1] / p[2] and abs(out[2] / p[2] - 1) <= 1e-3
