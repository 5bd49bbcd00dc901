"""Thin Python binding over the C ABI (argument marshalling only).

Tensors are torch tensors on the GPU; their data pointers and the current
torch stream are handed to the library, which enqueues its kernels and
returns.  Outputs the caller does not pass are allocated with torch on the
input's device.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

DFT_FFT = 0x0
DFT_MFMA_BF16X3 = 0x1
DFT_MFMA_FP16 = 0x2
DFT_MFMA_FP16X2 = 0x3
FIT_COLD = 0x00
FIT_WARM_MLP = 0x10
FIT_NONE = 0x20
FIT_FANO = 0x30

FIT_CONVERGED, FIT_MAX_ITER, FIT_SINGULAR, FIT_FALLBACK = 0, 1, 2, 3
TUNE_LM_CHUNK = 1
TUNE_LM_LANES = 2
TUNE_FFT_BLOCKS = 3
MLP_NPARAMS = 123396
MLP_IN = 220


def _dev_ptr(t, dtype, shape, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


SAMPLES_INT16, SAMPLES_INT8 = 0, 1


class Plan:
    """Plan for frames of `frame_len` samples (int16, or int8 with
    sample_type="int8") and `len(tooth_bins)` teeth."""

    def __init__(self, frame_len: int, fs: float, tooth_bins, ref_spectrum,
                 sample_type: str = "int16"):
        self._lib = _lib.load()
        bins = np.ascontiguousarray(np.asarray(tooth_bins), dtype=np.int32)
        ref = np.ascontiguousarray(np.asarray(ref_spectrum), dtype=np.float32)
        if bins.ndim != 1 or ref.shape != bins.shape:
            raise ValueError("tooth_bins and ref_spectrum must be 1-D of equal length")
        if sample_type not in ("int16", "int8"):
            raise ValueError("sample_type must be 'int16' or 'int8'")
        handle = ctypes.c_void_p()
        st = self._lib.cg_create_plan_ex(int(frame_len), float(fs),
                                         bins.ctypes.data_as(_lib._pi32), int(bins.shape[0]),
                                         ref.ctypes.data_as(_lib._pf32),
                                         SAMPLES_INT8 if sample_type == "int8" else SAMPLES_INT16,
                                         ctypes.byref(handle))
        _lib.check(st, "cg_create_plan_ex")
        self.sample_type = sample_type
        self.sample_dtype = torch.int8 if sample_type == "int8" else torch.int16
        self.np_dtype = np.int8 if sample_type == "int8" else np.int16
        self._h = handle
        self.frame_len = int(frame_len)
        self.fs = float(fs)
        self.n_teeth = int(bins.shape[0])
        self.tooth_bins = bins.copy()

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.cg_destroy_plan(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- plan state -------------------------------------------------------
    def set_reference(self, ref_spectrum):
        ref = np.ascontiguousarray(np.asarray(ref_spectrum), dtype=np.float32)
        if ref.shape != (self.n_teeth,):
            raise ValueError("reference length must equal n_teeth")
        _lib.check(self._lib.cg_set_reference(self._h, ref.ctypes.data_as(_lib._pf32)),
                   "cg_set_reference")

    def info(self):
        n, k, fs = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _lib.check(self._lib.cg_plan_info(self._h, ctypes.byref(n), ctypes.byref(k),
                                          ctypes.byref(fs)), "cg_plan_info")
        return n.value, k.value, fs.value

    def set_tuning(self, knob: int, value: int):
        _lib.check(self._lib.cg_set_tuning(self._h, int(knob), int(value)), "cg_set_tuning")

    def workspace_bytes(self, n_frames: int) -> int:
        b = ctypes.c_size_t()
        _lib.check(self._lib.cg_workspace_bytes(self._h, int(n_frames), ctypes.byref(b)),
                   "cg_workspace_bytes")
        return b.value

    # -- hot path -----------------------------------------------------------
    def _frames(self, frames):
        if frames.dim() != 2 or frames.shape[1] != self.frame_len:
            raise ValueError(f"frames must be [n, {self.frame_len}]")
        nf = int(frames.shape[0])
        return nf, _dev_ptr(frames, self.sample_dtype, (nf, self.frame_len), "frames")

    def process(self, frames, params=None, iters=None, status=None, chi2=None, teeth=None,
                y=None, flags: int = 0, workspace=None, want=("params",)):
        """Run the whole path on a batch.  Outputs named in `want` and not
        passed in are allocated; returns a dict of every output written."""
        nf, fp = self._frames(frames)
        dev = frames.device
        k = self.n_teeth
        out = {}

        def alloc(name, given, shape, dtype):
            if given is None and name in want:
                given = torch.empty(shape, dtype=dtype, device=dev)
            if given is not None:
                out[name] = given
            return given

        fit = flags & 0xF0
        if fit == FIT_NONE:
            params = None
        else:
            params = alloc("params", params, (nf, 4), torch.float32)
        iters = alloc("iters", iters, (nf,), torch.int32)
        status = alloc("status", status, (nf,), torch.int32)
        chi2 = alloc("chi2", chi2, (nf,), torch.float32)
        teeth = alloc("teeth", teeth, (nf, k), torch.float32)
        y = alloc("y", y, (nf, k), torch.float32)
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous GPU tensor")
            ws_ptr = ctypes.c_void_p(workspace.data_ptr())
            ws_bytes = workspace.numel() * workspace.element_size()
        st = self._lib.cg_process_batch_ex(
            self._h, fp, nf,
            _dev_ptr(params, torch.float32, (nf, 4), "params") if params is not None else None,
            _dev_ptr(iters, torch.int32, (nf,), "iters"),
            _dev_ptr(status, torch.int32, (nf,), "status"),
            _dev_ptr(chi2, torch.float32, (nf,), "chi2"),
            _dev_ptr(teeth, torch.float32, (nf, k), "teeth"),
            _dev_ptr(y, torch.float32, (nf, k), "y"),
            int(flags), ws_ptr, int(ws_bytes), _stream(dev))
        _lib.check(st, "cg_process_batch_ex")
        return out

    def process_static(self, frames, params=None, iters=None, status=None, chi2=None,
                       flags: int = 0):
        """Whole path with the library's fixed scratch array as workspace
        (cg_process_batch_static: no device allocation inside the call).
        Outputs not passed are allocated here, before the call."""
        nf, fp = self._frames(frames)
        dev = frames.device
        if params is None:
            params = torch.empty((nf, 4), dtype=torch.float32, device=dev)
        st = self._lib.cg_process_batch_static(
            self._h, fp, nf, _dev_ptr(params, torch.float32, (nf, 4), "params"),
            _dev_ptr(iters, torch.int32, (nf,), "iters"),
            _dev_ptr(status, torch.int32, (nf,), "status"),
            _dev_ptr(chi2, torch.float32, (nf,), "chi2"), int(flags), _stream(dev))
        _lib.check(st, "cg_process_batch_static")
        return params

    def process_batch(self, frames, params):
        """Plain entry point: writes params [n, 4] (centre, width, depth, baseline)."""
        nf, fp = self._frames(frames)
        st = self._lib.cg_process_batch(self._h, fp, nf,
                                        _dev_ptr(params, torch.float32, (nf, 4), "params"),
                                        _stream(frames.device))
        _lib.check(st, "cg_process_batch")
        return params

    def teeth(self, frames, flags: int = DFT_FFT, want_mag=True, want_y=True, out_mag=None,
              out_y=None):
        nf, fp = self._frames(frames)
        dev = frames.device
        mag, y = out_mag, out_y
        if mag is None and want_mag:
            mag = torch.empty((nf, self.n_teeth), dtype=torch.float32, device=dev)
        if y is None and want_y:
            y = torch.empty((nf, self.n_teeth), dtype=torch.float32, device=dev)
        st = self._lib.cg_teeth(self._h, fp, nf,
                                _dev_ptr(mag, torch.float32, (nf, self.n_teeth), "teeth"),
                                _dev_ptr(y, torch.float32, (nf, self.n_teeth), "y"),
                                int(flags), _stream(dev))
        _lib.check(st, "cg_teeth")
        return mag, y

    def reference_from_frames(self, ref_frames):
        nf, fp = self._frames(ref_frames)
        out = torch.empty((self.n_teeth,), dtype=torch.float32, device=ref_frames.device)
        st = self._lib.cg_reference_from_frames(self._h, fp, nf,
                                                ctypes.c_void_p(out.data_ptr()),
                                                _stream(ref_frames.device))
        _lib.check(st, "cg_reference_from_frames")
        return out

    def init_spectra(self, y, want_median=False, out_p0=None):
        nf = int(y.shape[0])
        yp = _dev_ptr(y, torch.float32, (nf, self.n_teeth), "y")
        p0 = out_p0 if out_p0 is not None else \
            torch.empty((nf, 4), dtype=torch.float32, device=y.device)
        _dev_ptr(p0, torch.float32, (nf, 4), "p0")
        med = torch.empty((nf, self.n_teeth), dtype=torch.float32, device=y.device) \
            if want_median else None
        st = self._lib.cg_init_spectra(self._h, yp, nf, ctypes.c_void_p(p0.data_ptr()),
                                       _dev_ptr(med, torch.float32, (nf, self.n_teeth), "median"),
                                       _stream(y.device))
        _lib.check(st, "cg_init_spectra")
        return p0, med

    def start_centres(self, y, out_p0=None):
        """The 7x7-median start centres alone (column 0 of out_p0 [n, 4]; the
        other columns are left as they are): the Fano fit's start."""
        nf = int(y.shape[0])
        if out_p0 is None:
            out_p0 = torch.zeros((nf, 4), dtype=torch.float32, device=y.device)
        yp = _dev_ptr(y, torch.float32, (nf, self.n_teeth), "y")
        pp = _dev_ptr(out_p0, torch.float32, (nf, 4), "p0")
        st = self._lib.cg_start_centres(self._h, yp, nf, pp, _stream(y.device))
        _lib.check(st, "cg_start_centres")
        return out_p0

    def init_spectra_listed(self, y, listed, out_p0):
        """Start points for the frames with listed[f] != 0 (int32 device
        tensor); the other rows of out_p0 are left as they are."""
        nf = int(y.shape[0])
        yp = _dev_ptr(y, torch.float32, (nf, self.n_teeth), "y")
        lp = _dev_ptr(listed, torch.int32, (nf,), "listed")
        pp = _dev_ptr(out_p0, torch.float32, (nf, 4), "p0")
        st = self._lib.cg_init_spectra_listed(self._h, yp, nf, lp, pp, _stream(y.device))
        _lib.check(st, "cg_init_spectra_listed")
        return out_p0

    def set_mlp(self, params, out_mean, out_std, noise_floor: float):
        """Install warm-start weights (flat float32 [MLP_NPARAMS])."""
        prm = np.ascontiguousarray(np.asarray(params), dtype=np.float32)
        if prm.shape != (MLP_NPARAMS,):
            raise ValueError(f"params must have {MLP_NPARAMS} values")
        mean = np.ascontiguousarray(np.asarray(out_mean), dtype=np.float32)
        std = np.ascontiguousarray(np.asarray(out_std), dtype=np.float32)
        if mean.shape != (4,) or std.shape != (4,):
            raise ValueError("out_mean and out_std must have 4 values")
        st = self._lib.cg_set_mlp(self._h, prm.ctypes.data_as(_lib._pf32),
                                  mean.ctypes.data_as(_lib._pf32), std.ctypes.data_as(_lib._pf32),
                                  float(noise_floor))
        _lib.check(st, "cg_set_mlp")

    def set_fano(self, width: float, asymmetry: float, depth_avg: float, scale_avg: float):
        """Fixed width and asymmetry and the averages of extent and scale of
        the paper's Fano fit (FIT_FANO)."""
        _lib.check(self._lib.cg_set_fano(self._h, float(width), float(asymmetry),
                                         float(depth_avg), float(scale_avg)), "cg_set_fano")

    def fit_fano(self, y, p0, max_iter: int = 20, out=None):
        """The Fano fit alone from start centres p0[:, 0]."""
        nf = int(y.shape[0])
        yp = _dev_ptr(y, torch.float32, (nf, self.n_teeth), "y")
        pp = _dev_ptr(p0, torch.float32, (nf, 4), "p0")
        dev = y.device
        if out is None:
            out = (torch.empty((nf, 4), dtype=torch.float32, device=dev),
                   torch.empty((nf,), dtype=torch.int32, device=dev),
                   torch.empty((nf,), dtype=torch.int32, device=dev),
                   torch.empty((nf,), dtype=torch.float32, device=dev))
        params, iters, status, chi2 = out
        st = self._lib.cg_fit_fano(self._h, yp, pp, nf, int(max_iter),
                                   _dev_ptr(params, torch.float32, (nf, 4), "params"),
                                   _dev_ptr(iters, torch.int32, (nf,), "iters"),
                                   _dev_ptr(status, torch.int32, (nf,), "status"),
                                   _dev_ptr(chi2, torch.float32, (nf,), "chi2"), _stream(dev))
        _lib.check(st, "cg_fit_fano")
        return params, iters, status, chi2

    def set_polish_iters(self, iters: int):
        """LM iterations from the network's start point in the learned warm
        start (default 2; 20, the cold start's cap, makes it a full fit)."""
        _lib.check(self._lib.cg_set_polish_iters(self._h, int(iters)), "cg_set_polish_iters")

    def mlp_infer(self, y, out=None):
        nf = int(y.shape[0])
        yp = _dev_ptr(y, torch.float32, (nf, self.n_teeth), "y")
        if out is None:
            out = torch.empty((nf, 4), dtype=torch.float32, device=y.device)
        st = self._lib.cg_mlp_infer(self._h, yp, nf, _dev_ptr(out, torch.float32, (nf, 4), "p0"),
                                    _stream(y.device))
        _lib.check(st, "cg_mlp_infer")
        return out

    def get_tuning(self, knob: int) -> int:
        v = ctypes.c_int32()
        _lib.check(self._lib.cg_get_tuning(self._h, int(knob), ctypes.byref(v)), "cg_get_tuning")
        return v.value

    def tuned_shape(self):
        """The plan's launch shape: fit lanes per spectrum, spectra per
        wavefront and FFT grid cap (0 = chosen automatically)."""
        return {"lm_lanes": self.get_tuning(TUNE_LM_LANES),
                "lm_chunk": self.get_tuning(TUNE_LM_CHUNK),
                "fft_blocks": self.get_tuning(TUNE_FFT_BLOCKS)}

    def autotune(self, frames, flags: int = 0):
        """Pick the fastest launch shape for these frames (see cg_autotune);
        returns (spectra per wavefront, ms per batch)."""
        nf, fp = self._frames(frames)
        chosen = ctypes.c_int32()
        best = ctypes.c_float()
        st = self._lib.cg_autotune(self._h, fp, nf, int(flags), None, 0, ctypes.byref(chosen),
                                   ctypes.byref(best))
        _lib.check(st, "cg_autotune")
        return chosen.value, best.value

    def median_filter(self, y, out=None):
        nf = int(y.shape[0])
        yp = _dev_ptr(y, torch.float32, (nf, self.n_teeth), "y")
        if out is None:
            out = torch.empty((nf, self.n_teeth), dtype=torch.float32, device=y.device)
        st = self._lib.cg_median_filter(self._h, yp, nf,
                                        _dev_ptr(out, torch.float32, (nf, self.n_teeth), "median"),
                                        _stream(y.device))
        _lib.check(st, "cg_median_filter")
        return out

    def start_points(self, median, out=None):
        nf = int(median.shape[0])
        mp = _dev_ptr(median, torch.float32, (nf, self.n_teeth), "median")
        if out is None:
            out = torch.empty((nf, 4), dtype=torch.float32, device=median.device)
        st = self._lib.cg_start_points(self._h, mp, nf, _dev_ptr(out, torch.float32, (nf, 4), "p0"),
                                       _stream(median.device))
        _lib.check(st, "cg_start_points")
        return out

    def fit_spectra(self, y, p0, max_iter: int = 20, out=None):
        nf = int(y.shape[0])
        yp = _dev_ptr(y, torch.float32, (nf, self.n_teeth), "y")
        pp = _dev_ptr(p0, torch.float32, (nf, 4), "p0")
        dev = y.device
        if out is None:
            out = (torch.empty((nf, 4), dtype=torch.float32, device=dev),
                   torch.empty((nf,), dtype=torch.int32, device=dev),
                   torch.empty((nf,), dtype=torch.int32, device=dev),
                   torch.empty((nf,), dtype=torch.float32, device=dev))
        params, iters, status, chi2 = out
        _dev_ptr(params, torch.float32, (nf, 4), "params")
        _dev_ptr(iters, torch.int32, (nf,), "iters")
        _dev_ptr(status, torch.int32, (nf,), "status")
        _dev_ptr(chi2, torch.float32, (nf,), "chi2")
        st = self._lib.cg_fit_spectra(self._h, yp, pp, nf, int(max_iter),
                                      ctypes.c_void_p(params.data_ptr()),
                                      ctypes.c_void_p(iters.data_ptr()),
                                      ctypes.c_void_p(status.data_ptr()),
                                      ctypes.c_void_p(chi2.data_ptr()), _stream(dev))
        _lib.check(st, "cg_fit_spectra")
        return params, iters, status, chi2


class Trainer:
    """Training state of the warm-start network (FP32 master weights, Adam
    moments, mini-batch buffers) on the GPU; every step runs in the library's
    kernels."""

    def __init__(self, batch: int, init_params):
        self._lib = _lib.load()
        init = np.ascontiguousarray(np.asarray(init_params), dtype=np.float32)
        if init.shape != (MLP_NPARAMS,):
            raise ValueError(f"init_params must have {MLP_NPARAMS} values")
        h = ctypes.c_void_p()
        st = self._lib.cg_mlp_trainer_create(int(batch), init.ctypes.data_as(_lib._pf32),
                                             ctypes.byref(h))
        _lib.check(st, "cg_mlp_trainer_create")
        self._h = h
        self.batch = int(batch)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.cg_mlp_trainer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _args(self, x, targets, weights, idx):
        n = int(x.shape[0])
        xp = _dev_ptr(x, torch.float32, (n, MLP_IN), "x")
        tp = _dev_ptr(targets, torch.float32, (n, 4), "targets")
        wp = _dev_ptr(weights, torch.float32, (n,), "weights") if weights is not None else None
        ip = _dev_ptr(idx, torch.int32, (self.batch,), "idx")
        return xp, tp, wp, ip

    def step(self, x, targets, weights, idx, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
             loss=None):
        xp, tp, wp, ip = self._args(x, targets, weights, idx)
        lp = _dev_ptr(loss, torch.float32, (1,), "loss") if loss is not None else None
        st = self._lib.cg_mlp_train_step(self._h, xp, tp, wp, ip, float(lr), float(beta1),
                                         float(beta2), float(eps), lp, _stream(x.device))
        _lib.check(st, "cg_mlp_train_step")

    def gradients(self, x, targets, weights, idx):
        xp, tp, wp, ip = self._args(x, targets, weights, idx)
        g = torch.empty((MLP_NPARAMS,), dtype=torch.float32, device=x.device)
        loss = torch.empty((1,), dtype=torch.float32, device=x.device)
        st = self._lib.cg_mlp_gradients(self._h, xp, tp, wp, ip, ctypes.c_void_p(g.data_ptr()),
                                        ctypes.c_void_p(loss.data_ptr()), _stream(x.device))
        _lib.check(st, "cg_mlp_gradients")
        return g, loss

    def params(self):
        out = np.empty(MLP_NPARAMS, dtype=np.float32)
        _lib.check(self._lib.cg_mlp_get_params(self._h, out.ctypes.data_as(_lib._pf32)),
                   "cg_mlp_get_params")
        return out


PIPE_KEEP_RESULTS = 0x1
PIPE_DRY_RUN = 0x2
PIPE_HOST_RING = 0x4
STATS_FIELDS = ("bursts", "frames", "bytes", "overflows", "seconds", "lat_p50_ms", "lat_p99_ms",
                "lat_max_ms", "bytes_per_s", "frames_per_s", "dev_lat_p50_ms", "dev_lat_p99_ms",
                "dev_lat_max_ms", "dev_span_p50_ms", "out_of_order", "launch_max_ms",
                "dispatch_pass_max_ms")


class RingFull(_lib.CombGpuError):
    pass


class Pipeline:
    """Multi-stream ring pipeline (see cg_pipeline_create).  `plans` and
    `fit_flags` per stream; in dry-run mode pass `n_streams` instead."""

    def __init__(self, plans=None, fit_flags=None, slots_per_stream=4, max_burst_frames=4096,
                 keep_results=False, dry_run_us_per_frame=None, n_streams=None, lanes=1,
                 host_ring=False):
        self._lib = _lib.load()
        opts = PIPE_KEEP_RESULTS if keep_results else 0
        if host_ring:
            opts |= PIPE_HOST_RING
        self.host_ring = bool(host_ring)
        if dry_run_us_per_frame is not None:
            opts |= PIPE_DRY_RUN
            ns = int(n_streams)
            arr_p = arr_f = None
            dry = float(dry_run_us_per_frame)
        else:
            ns = len(plans)
            arr_p = (ctypes.c_void_p * ns)(*[p._h.value for p in plans])
            arr_f = (ctypes.c_uint32 * ns)(*[int(f) for f in fit_flags])
            dry = 0.0
        self._plans = plans  # keep alive
        h = ctypes.c_void_p()
        st = self._lib.cg_pipeline_create_ex(ns, arr_p, arr_f, int(slots_per_stream),
                                             int(max_burst_frames), opts, int(lanes), dry,
                                             ctypes.byref(h))
        _lib.check(st, "cg_pipeline_create_ex")
        self.frame_len = [p.frame_len for p in plans] if plans is not None else None
        self.np_dtype = [p.np_dtype for p in plans] if plans is not None else None
        self._h = h
        self.n_streams = ns
        self.max_burst = int(max_burst_frames)
        self.slots = int(slots_per_stream)
        # the source of each slot's queued copy stays referenced until the
        # slot is taken again (its burst has then completed)
        self._held = [dict() for _ in range(ns)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.cg_pipeline_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def acquire(self, stream: int):
        """Returns (slot, device pointer of the slot's frame buffer) or raises RingFull."""
        slot = ctypes.c_int32()
        ptr = ctypes.c_void_p()
        st = self._lib.cg_pipeline_acquire(self._h, int(stream), ctypes.byref(slot),
                                           ctypes.byref(ptr))
        if st == -9:
            raise RingFull(st, "cg_pipeline_acquire")
        _lib.check(st, "cg_pipeline_acquire")
        return slot.value, ptr.value

    def acquire_host(self, stream: int):
        """Host ring: (slot, numpy view [max_burst_frames, frame_len] of the
        slot's pinned host buffer, in the plan's sample type) or raises
        RingFull."""
        if not self.host_ring:
            raise ValueError("acquire_host needs a pipeline created with host_ring=True")
        slot, ptr = self.acquire(stream)
        dt = np.dtype(self.np_dtype[int(stream)])
        n = self.max_burst * self.frame_len[int(stream)] * dt.itemsize
        buf = (ctypes.c_uint8 * n).from_address(ptr)
        return slot, np.frombuffer(buf, dtype=dt).reshape(self.max_burst, -1)

    def publish(self, stream: int, slot: int, n_frames: int, seq: int):
        _lib.check(self._lib.cg_pipeline_publish(self._h, int(stream), int(slot), int(n_frames),
                                                 int(seq)), "cg_pipeline_publish")

    def put(self, stream: int, frames, seq: int):
        """Copy a burst (torch int16 tensor on the GPU or pinned CPU tensor,
        [n, frame_len], contiguous; with the host ring a host numpy array or
        CPU tensor, copied into the ring on this thread) into a free slot and
        publish it.  Raises RingFull when the stream has no free slot."""
        s = int(stream)
        want_np = np.dtype(self.np_dtype[s]) if self.np_dtype else np.dtype(np.int16)
        want_t = torch.int8 if want_np == np.int8 else torch.int16
        if isinstance(frames, np.ndarray):
            if not self.host_ring:
                raise ValueError("numpy sources need a host-ring pipeline")
            if frames.dtype != want_np or frames.ndim != 2 or not frames.flags.c_contiguous \
                    or frames.shape[1] != self.frame_len[s]:
                raise ValueError(f"frames must be a C-contiguous {want_np} array [n, frame_len]")
            ptr, nfr = frames.ctypes.data, int(frames.shape[0])
        else:
            if not isinstance(frames, torch.Tensor) or frames.dtype != want_t or \
                    frames.dim() != 2 or not frames.is_contiguous() or \
                    frames.shape[1] != self.frame_len[s]:
                raise ValueError(f"frames must be a contiguous {want_t} tensor [n, frame_len]")
            if self.host_ring and frames.is_cuda:
                raise ValueError("a host-ring pipeline takes host frames")
            ptr, nfr = frames.data_ptr(), int(frames.shape[0])
        slot = ctypes.c_int32(-1)
        st = self._lib.cg_pipeline_put(self._h, int(stream), ctypes.c_void_p(ptr), nfr, int(seq),
                                       ctypes.byref(slot))
        if st == -9:
            raise RingFull(st, "cg_pipeline_put")
        _lib.check(st, "cg_pipeline_put")
        if not self.host_ring:
            self._held[int(stream)][slot.value] = frames

    def read(self, stream: int):
        """Oldest completed burst of `stream`: (seq, params [n,4], status [n]) or None."""
        params = np.empty((self.max_burst, 4), dtype=np.float32)
        status = np.empty(self.max_burst, dtype=np.int32)
        n = ctypes.c_int32()
        seq = ctypes.c_int64()
        st = self._lib.cg_pipeline_read(self._h, int(stream), params.ctypes.data_as(_lib._pf32),
                                        status.ctypes.data_as(_lib._pi32), self.max_burst,
                                        ctypes.byref(n), ctypes.byref(seq))
        if st == -8 and n.value == 0:
            return None
        _lib.check(st, "cg_pipeline_read")
        return seq.value, params[:n.value].copy(), status[:n.value].copy()

    def drain(self, timeout_ms: int = 60000):
        _lib.check(self._lib.cg_pipeline_drain(self._h, int(timeout_ms)), "cg_pipeline_drain")
        self._held = [dict() for _ in range(self.n_streams)]

    def stats(self):
        out = (ctypes.c_double * len(STATS_FIELDS))()
        _lib.check(self._lib.cg_pipeline_stats(self._h, out, len(STATS_FIELDS)),
                   "cg_pipeline_stats")
        return dict(zip(STATS_FIELDS, list(out)))


def psd_band(seg_len: int, fs: float, f_lo: float, f_hi: float):
    """(k_lo, n_bins) of the band [f_lo, f_hi] Hz for segments of seg_len."""
    lib = _lib.load()
    k_lo, nb = ctypes.c_int32(), ctypes.c_int32()
    _lib.check(lib.cg_psd_band(int(seg_len), float(fs), float(f_lo), float(f_hi),
                               ctypes.byref(k_lo), ctypes.byref(nb)), "cg_psd_band")
    return k_lo.value, nb.value


def psd_welch(series, fs: float, seg_len: int, k_lo: int, n_bins: int, workspace=None):
    """Welch density of a device float32 series at bins k_lo .. k_lo+n_bins-1
    (device float64 tensor), see cg_psd_welch."""
    lib = _lib.load()
    if not isinstance(series, torch.Tensor) or not series.is_cuda or series.dtype != torch.float32 \
            or series.dim() != 1 or not series.is_contiguous():
        raise ValueError("series must be a contiguous 1-D float32 tensor on the GPU")
    n = int(series.shape[0])
    need = ctypes.c_size_t()
    _lib.check(lib.cg_psd_workspace_bytes(n, int(seg_len), int(n_bins), ctypes.byref(need)),
               "cg_psd_workspace_bytes")
    if workspace is None:
        workspace = torch.empty(need.value, dtype=torch.uint8, device=series.device)
    out = torch.empty(int(n_bins), dtype=torch.float64, device=series.device)
    st = lib.cg_psd_welch(ctypes.c_void_p(series.data_ptr()), n, float(fs), int(seg_len),
                          int(k_lo), int(n_bins), ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(workspace.data_ptr()), int(workspace.numel()),
                          _stream(series.device))
    _lib.check(st, "cg_psd_welch")
    return out


def resonance_fit(psd, f_first: float, df: float, max_iter: int = 100, tol: float = 1e-9):
    """Fit of the mechanical resonance to a device float64 PSD band: device
    float64 [7] = ln A, f0, Q, ln B, chi2, iterations, status."""
    lib = _lib.load()
    if not isinstance(psd, torch.Tensor) or not psd.is_cuda or psd.dtype != torch.float64 \
            or psd.dim() != 1 or not psd.is_contiguous():
        raise ValueError("psd must be a contiguous 1-D float64 tensor on the GPU")
    out = torch.empty(7, dtype=torch.float64, device=psd.device)
    st = lib.cg_resonance_fit(ctypes.c_void_p(psd.data_ptr()), int(psd.shape[0]), float(f_first),
                              float(df), int(max_iter), float(tol),
                              ctypes.c_void_p(out.data_ptr()), _stream(psd.device))
    _lib.check(st, "cg_resonance_fit")
    return out
