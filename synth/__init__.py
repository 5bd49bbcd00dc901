"""Seeded synthetic comb-spectroscopy streams.

This package only produces inputs: digitised interferogram frames (int16), a
reference frame and the ground-truth dip parameters used to synthesise them.
It holds none of the processing method's arithmetic (no transform of the
frames, no tooth extraction, no normalisation and no fit); both the FP64
oracle and the GPU path consume what it produces.
"""

from .comb import (
    StreamSpec,
    Batch,
    tooth_bins_paper_c1,
    tooth_bins_interleaved,
    tooth_bins_paper_2200,
    make_batch,
    make_lorentzian_spectra,
    make_displacement,
    spec_tiny,
    spec_paper_rate,
    spec_precision,
    spec_learned,
    spec_multistream,
    spec_fano,
    spec_paper8,
)

__all__ = [
    "StreamSpec",
    "Batch",
    "tooth_bins_paper_c1",
    "tooth_bins_interleaved",
    "tooth_bins_paper_2200",
    "make_batch",
    "make_lorentzian_spectra",
    "make_displacement",
    "spec_tiny",
    "spec_paper_rate",
    "spec_precision",
    "spec_learned",
    "spec_multistream",
    "spec_fano",
    "spec_paper8",
]
