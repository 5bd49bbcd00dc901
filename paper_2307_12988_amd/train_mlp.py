"""Train the learned warm start on spectra and fits the method itself generates.

    python -m paper_2307_12988_amd.train_mlp [--samples 1048576] [--epochs 20]
        [--out paper_2307_12988_amd/data/warmstart_learned.npz]

1. Synthetic frames of the warm-start training distribution (centre
   mid +- 40 teeth, FWHM 3..20, depth 0.1..0.9, SNR 15..50 dB, linear baseline
   tilt +-5 %, each drifting continuously; 2048 samples, 220 teeth), seed 3;
   hold-out seed 4.
2. The GPU path turns them into normalised spectra and cold-start
   Levenberg-Marquardt fits; converged fits of a dip inside the comb
   (0 <= c <= K-1, 1 < w < K/4, 0.02 < d <= 1.2) are the labels (the others get
   weight 0).
3. Calibration constants, computed on the host from those GPU outputs: the
   per-output mean and standard deviation of the labels, and the noise floor
   (median RMS residual sqrt(chi2 / (K - 4)) of the converged fits).
4. Adam (betas 0.9/0.999, batch 1024, learning rate 1e-3 decayed along a
   cosine to 1e-5 over the run) on the weighted MSE of the standardised
   labels, He-normal initial weights and per-epoch shuffles drawn from numpy's
   PCG64 with fixed seeds and passed to the kernels.
5. Hold-out report: warm start (network + 2-iteration polish + fallback)
   against the cold start on the same frames.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

DEFAULT_OUT = os.path.join(HERE, "data", "warmstart_learned.npz")
BATCH_FRAMES = 65536


def _gen(args):
    spec, nf, seed, b = args
    bt = synth.make_batch(spec, nf, seed=seed, batch_index=b)
    return b, bt.frames, bt.ref_frames


def he_init(seed: int):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, flat layout."""
    from .plan import MLP_NPARAMS
    rng = np.random.default_rng([int(seed), 11])
    parts = []
    for (fo, fi) in ((256, 220), (256, 256), (4, 256)):
        parts.append(rng.standard_normal(fo * fi) * np.sqrt(2.0 / fi))
        parts.append(np.zeros(fo))
    p = np.concatenate(parts).astype(np.float32)
    assert p.shape == (MLP_NPARAMS,)
    return p


def label_set(plan, spec, n_samples, seed, dev, workers=8, log=print):
    """GPU normalised spectra, cold-start fits and statuses for n_samples frames."""
    import torch
    n_batches = (n_samples + BATCH_FRAMES - 1) // BATCH_FRAMES
    ys, ps, sts, c2s = [], [], [], []
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        jobs = [(spec, BATCH_FRAMES, seed, b) for b in range(n_batches)]
        for b, frames, ref_frames in ex.map(_gen, jobs):
            fr = torch.from_numpy(frames).to(dev)
            if b == 0:
                ref = plan.reference_from_frames(torch.from_numpy(ref_frames).to(dev))
                plan.set_reference(ref.cpu().numpy())
            out = plan.process(fr, want=("params", "status", "chi2", "y"))
            ys.append(out["y"])
            ps.append(out["params"])
            sts.append(out["status"])
            c2s.append(out["chi2"])
            log(f"  batch {b + 1}/{n_batches}")
    y = torch.cat(ys)[:n_samples].contiguous()
    return (y, torch.cat(ps)[:n_samples].contiguous(), torch.cat(sts)[:n_samples].contiguous(),
            torch.cat(c2s)[:n_samples].contiguous())


def calibration(params, status, chi2, k):
    """Label mean/std over kept fits and the noise floor (host).  Kept: the
    cold-start fit converged to a dip inside the comb (0 <= c <= K-1,
    1 < w < K/4, 0.02 < d <= 1.2)."""
    p = params.cpu().numpy().astype(np.float64)
    st = status.cpu().numpy()
    c2 = chi2.cpu().numpy().astype(np.float64)
    ok = (st == 0) & (p[:, 0] >= 0) & (p[:, 0] <= k - 1) & (p[:, 1] > 1.0) & \
        (p[:, 1] < 0.25 * k) & (p[:, 2] > 0.02) & (p[:, 2] <= 1.2) & \
        np.all(np.isfinite(p), axis=1)
    mean = p[ok].mean(axis=0)
    std = p[ok].std(axis=0)
    noise = float(np.median(np.sqrt(np.maximum(c2[ok], 0.0) / (k - 4))))
    return mean.astype(np.float32), std.astype(np.float32), noise, ok


def train(samples=1 << 20, epochs=20, batch=1024, lr=1e-3, holdout=1 << 16, out=DEFAULT_OUT,
          log=print, workers=8):
    import torch

    from . import Plan, Trainer, FIT_WARM_MLP

    dev = torch.device("cuda:0")
    spec = synth.spec_learned()
    k = spec.k
    plan = Plan(spec.n, spec.fs, spec.bins, np.ones(k, dtype=np.float32))
    t0 = time.perf_counter()
    log(f"labelling {samples} training frames ...")
    y, lab, st, c2 = label_set(plan, spec, samples, 3, dev, workers, log)
    mean, std, noise, ok = calibration(lab, st, c2, k)
    log(f"  converged {ok.mean():.4f}, mean {mean}, std {std}, noise floor {noise:.4g}, "
        f"{time.perf_counter() - t0:.1f} s")
    z = ((lab.cpu().numpy() - mean) / std).astype(np.float32)
    zt = torch.from_numpy(z).to(dev)
    wt = torch.from_numpy(ok.astype(np.float32)).to(dev)
    tr = Trainer(batch, he_init(5))
    rng = np.random.default_rng([5, 13])
    loss = torch.zeros((1,), dtype=torch.float32, device=dev)
    curve = []
    steps = samples // batch
    t1 = time.perf_counter()
    total = epochs * steps
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(samples).astype(np.int32)).to(dev)
        acc = 0.0
        for s in range(steps):
            frac = (ep * steps + s) / max(1, total - 1)
            lr_t = 1e-5 + 0.5 * (lr - 1e-5) * (1.0 + np.cos(np.pi * frac))
            tr.step(y, zt, wt, perm[s * batch:(s + 1) * batch], lr=lr_t, loss=loss)
            if s % 64 == 63:
                acc += float(loss.item())
        curve.append(acc / max(1, steps // 64))
        log(f"  epoch {ep + 1}/{epochs}: mean loss {curve[-1]:.5f}")
    torch.cuda.synchronize(dev)
    train_s = time.perf_counter() - t1
    params = tr.params()
    tr.close()

    # hold-out: warm start against cold start on the same frames
    plan.set_mlp(params, mean, std, noise)
    rep = holdout_report(plan, spec, holdout, dev, log)
    rep.update({"train_seconds": train_s, "epochs": epochs, "samples": samples,
                "loss_curve": curve, "noise_floor": noise, "converged_label_frac": float(ok.mean())})
    if out:
        os.makedirs(os.path.dirname(out), exist_ok=True)
        np.savez(out, params=params, out_mean=mean, out_std=std, noise_floor=np.float32(noise),
                 report=json.dumps(rep))
        log(f"wrote {out}")
    plan.close()
    return params, mean, std, noise, rep


def holdout_report(plan, spec, n, dev, log=print):
    import torch

    from . import FIT_WARM_MLP

    bt = synth.make_batch(spec, n, seed=4)
    fr = torch.from_numpy(bt.frames).to(dev)
    cold = plan.process(fr, want=("params", "iters", "status", "y"))
    warm = plan.process(fr, flags=FIT_WARM_MLP, want=("params", "iters", "status"))
    p_net = plan.mlp_infer(cold["y"]).cpu().numpy()
    torch.cuda.synchronize(dev)
    reps = 5
    times = {}
    for name, flags in (("cold", 0), ("warm", FIT_WARM_MLP)):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            plan.process(fr, flags=flags, want=("params",))
        ev[1].record()
        torch.cuda.synchronize(dev)
        times[name] = ev[0].elapsed_time(ev[1]) / reps
    pc, pw = cold["params"].cpu().numpy(), warm["params"].cpu().numpy()
    sc, sw = cold["status"].cpu().numpy(), warm["status"].cpu().numpy()
    conv = sc == 0
    err = np.abs(pw[:, 0] - pc[:, 0]) / np.abs(pc[:, 1])
    net_err = np.abs(p_net - pc) / np.abs(pc[:, 1:2])
    rep = {
        "network_vs_cold_median_err_fwhm": [float(v) for v in np.median(net_err[conv], axis=0)],
        "frames": int(n),
        "cold_ms_per_batch": times["cold"], "warm_ms_per_batch": times["warm"],
        "speedup": times["cold"] / times["warm"],
        "cold_mean_iters": float(cold["iters"].float().mean().item()),
        "warm_mean_iters": float(warm["iters"].float().mean().item()),
        "fallback_frac": float(np.mean(sw == 3)),
        "centre_vs_cold_within_1e-3_fwhm": float(np.mean(err[conv] <= 1e-3)),
        "centre_vs_cold_median_fwhm": float(np.median(err[conv])),
        "centre_vs_truth_rms_fwhm_cold": float(np.sqrt(np.mean(((pc[:, 0] - bt.centre) / bt.width) ** 2))),
        "centre_vs_truth_rms_fwhm_warm": float(np.sqrt(np.mean(((pw[:, 0] - bt.centre) / bt.width) ** 2))),
    }
    log(json.dumps(rep))
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=1 << 20)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--holdout", type=int, default=1 << 16)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--workers", type=int, default=8)
    a = ap.parse_args()
    train(a.samples, a.epochs, a.batch, a.lr, a.holdout, a.out,
          log=lambda m: print(m, flush=True), workers=a.workers)


if __name__ == "__main__":
    main()
