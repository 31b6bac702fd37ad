"""MI355X-native delay-and-sum ultrasound beamformer (gfx950 HIP kernels).

The library ``libdas.so`` (C ABI in ``include/das.h``) holds the whole hot
path; this package is its thin Python binding.
"""

from .das import Params, Plan, beamform, tx_plane_wave, tile_order, iq_dtype_code, kernel_variants, \
    choose_kernel_variant  # noqa: F401

__version__ = "0.1.0"
