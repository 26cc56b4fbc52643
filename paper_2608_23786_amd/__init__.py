"""MI355X-native Monte Carlo KBC lattice Boltzmann library (arXiv 2608.23786 hot path).

The compute path is the HIP library ``libmclbm.so`` behind the C ABI in
``include/mclbm.h``; this package only marshals arguments to it.
"""
from ._lib import MclbmError, SampleDesc, lib  # noqa: F401
from .ensemble import (RECORD_FIELDS, Ensemble, EnsembleKE, Sample, ensemble_moments, eoc_slope,  # noqa: F401
                       omega, sample_error, stream_copy, w1_1pt)
