"""MI355X (gfx950) comb-spectroscopy hot path: int16 frames -> real FFT ->
comb-tooth amplitudes -> division by the reference -> 7x7 median start point
-> Levenberg-Marquardt Lorentzian fit, as hand-written HIP kernels behind the
C ABI in include/combgpu.h.  This package is the thin Python binding."""

from ._lib import CombGpuError, load, header_functions, LIB_PATH
from .plan import (psd_band, psd_welch, resonance_fit, SAMPLES_INT16, SAMPLES_INT8, Plan, Trainer, Pipeline, RingFull, STATS_FIELDS, MLP_NPARAMS, MLP_IN, DFT_FFT, DFT_MFMA_BF16X3, DFT_MFMA_FP16, DFT_MFMA_FP16X2, FIT_COLD,
                   FIT_WARM_MLP, FIT_NONE, FIT_FANO, FIT_CONVERGED, FIT_MAX_ITER, FIT_SINGULAR, FIT_FALLBACK,
                   TUNE_LM_CHUNK, TUNE_LM_LANES, TUNE_FFT_BLOCKS)

__all__ = ["psd_band", "psd_welch", "resonance_fit", "SAMPLES_INT16", "SAMPLES_INT8", "Pipeline", "RingFull", "STATS_FIELDS", "Trainer", "MLP_NPARAMS", "MLP_IN", "CombGpuError", "load", "header_functions", "LIB_PATH", "Plan", "DFT_FFT",
           "DFT_MFMA_BF16X3", "DFT_MFMA_FP16", "DFT_MFMA_FP16X2", "FIT_COLD", "FIT_WARM_MLP",
           "FIT_NONE", "FIT_FANO", "FIT_CONVERGED", "FIT_MAX_ITER", "FIT_SINGULAR", "FIT_FALLBACK",
           "TUNE_LM_CHUNK", "TUNE_LM_LANES", "TUNE_FFT_BLOCKS"]
