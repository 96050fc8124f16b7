"""Seeded synthetic inputs (scan pointing, HEALPix RING pixels, sky, 1/f noise).

Shared by the oracle and the GPU path as their common input source; holds no
step of the destriping method itself.
"""
from .configs import Problem, make_problem, workload, realizations, gaussian_sky, signal_timelines  # noqa: F401
from .healpix_ring import ang2pix_ring, ang2pix_ring_z, pix2ang_ring, nside2npix  # noqa: F401
from .scan import ScanSpec, pointing  # noqa: F401
