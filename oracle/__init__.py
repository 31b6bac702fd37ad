"""FP64 CPU oracle for delay-and-sum (DAS) beamforming.  TEST INFRASTRUCTURE.

Only the tests, the smoke check of ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product path (the HIP
library and its Python binding) never imports, calls or links anything here,
and nothing here imports the product path.

Contents
--------
``das``              the defining DAS sum written out in complex128 (paper
                     Sec. 2.1 and Sec. 4.3; linear interpolation and f-number
                     apodization from Sec. 4.1).
``tx_plane_wave``    per-voxel plane-wave arrival times (the precomputed
                     transmit table of Sec. 3.3 step 3 / Sec. 4.3).
``apodization``      the f-number receive window (Tukey on the normalised
                     lateral distance; the paper names only the f-number).
``das_scalar``       an independent pure-Python scalar implementation (math
                     module only) used to pin ``das`` by brute force.
``accounting``       the paper's throughput (Eq. 1) and memory (Eq. 2,
                     Table 4) arithmetic.
"""

from .das_oracle import das, tx_plane_wave, apodization, tukey, nrmse_db, peak_err_db  # noqa: F401
from .brute import das_scalar  # noqa: F401
from . import accounting  # noqa: F401
