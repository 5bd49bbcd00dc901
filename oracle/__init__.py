"""FP64 CPU oracle of the comb-spectroscopy hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
statement of what the processing method computes, written from the paper's
"Data Capture and Processing" section.  It is imported only by the tests, by
the smoke check and by the CPU-baseline leg of the benchmark; the product path
(the HIP library and its Python binding) never imports, calls or falls back to
it, and it shares no code, tables or constants with that path.

Modules
-------
dft          ingest cast, DFT at the comb-tooth bins, magnitude, reference average
normalize    division by the reference spectrum
initializer  7x7 median filter over the (frame, tooth) image and the start point
lm           Levenberg-Marquardt fit of the Lorentzian cavity dip
fano         projected Levenberg-Marquardt fit of the asymmetric Fano dip
mlp          FP64 forward/backward of the warm-start network
psd          displacement power spectral density and the mechanical resonance fit
pipeline     the steps above chained for a batch of frames

Every function names the passage it follows.  Where the paper is silent the
reading taken is stated in the docstring.
"""

from .dft import frames_to_float, dft_at_bins, tooth_magnitudes, reference_spectrum, full_dft
from .normalize import normalize
from .initializer import median7x7, initial_guess
from .lm import lorentzian, lorentzian_jacobian, lm_fit, lm_fit_batch, chi2_at
from .pipeline import process_batch, process_batch_fano
from .fano import fano, fano_jacobian, fano_fit, fano_fit_batch, fano_box, chi2_fano

__all__ = [
    "frames_to_float",
    "dft_at_bins",
    "tooth_magnitudes",
    "reference_spectrum",
    "full_dft",
    "normalize",
    "median7x7",
    "initial_guess",
    "lorentzian",
    "lorentzian_jacobian",
    "lm_fit",
    "lm_fit_batch",
    "chi2_at",
    "process_batch",
    "process_batch_fano",
    "fano",
    "fano_jacobian",
    "fano_fit",
    "fano_fit_batch",
    "fano_box",
    "chi2_fano",
]
