"""CPU FP64 oracle of the FFT momentum power spectrum estimator.

TEST INFRASTRUCTURE: only tests/, the smoke check in __graft_entry__ and the
CPU-baseline leg of bench.py may import or run anything in this package.  The
GPU product path never calls it and shares no code with it.
"""
from .estimator import (  # noqa: F401
    FLAG_BULKFLOW_SUBTRACT, FLAG_NO_DECONVOLVE, FLAG_NO_SHOTNOISE, Spectra,
    assign, assign_cells, bin_modes, cell_and_fraction, default_bin_index, edge_thresholds,
    edges_bin_index, estimate, fourier_fields, mode_quantities, moments)
from . import bl3, bl3_quadratic  # noqa: F401
from .anisotropic import estimate_mu, mu_bin, unit_axis  # noqa: F401
from . import bspline, subcubes  # noqa: F401
