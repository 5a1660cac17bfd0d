"""MI355X-native FFT estimator of cosmic momentum power spectra.

Binds libmps.so (include/mps.h): BL3 assignment of rho and rho v to a
periodic grid, 3D real-to-complex FFTs, window deconvolution, shot-noise and
optional bulk-flow removal, and |k|-shell binning of P_pp, P_theta-theta and
P_delta-theta, all in HIP kernels for gfx950.  torch supplies device memory and
streams only.
"""
from .api import Plan, Server, estimate, estimate_batch, spt_one_loop  # noqa: F401
from ._lib import MpsError  # noqa: F401
