"""Seeded synthetic inputs for the delay-and-sum beamformer and its oracle.

This package is the only code shared by the GPU path's tests/bench and the
FP64 oracle.  It builds what an acquisition would hand a beamformer: array
geometry, a reconstruction grid, a transmit sequence (angles only) and complex
IQ channel data echoed by seeded point-scatterer phantoms.  It contains none
of the beamforming arithmetic (no receive delays on a grid, no apodization, no
interpolation, no summation over elements).

The echo model is a forward simulator: each scatterer is an ideal point
reflector that returns a Gaussian-modulated pulse delayed by its own
round-trip time (plane-wave transmit, spherical receive), with no spreading
loss, attenuation or element directivity.
"""

from .geometry import linear_array, matrix_array, grid_2d, grid_3d  # noqa: F401
from .echo import echo_iq, echo_iq_numpy, echo_iq_gpu, plane_wave_normals  # noqa: F401
from .configs import make_config, volume_phantom, CONFIGS  # noqa: F401
