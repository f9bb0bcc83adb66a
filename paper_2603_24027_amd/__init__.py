"""MI355X-native time-reversible FDTD gradient with compressed interface storage.

The compute path is the HIP library ``libfdtd_mi355x.so`` (include/fdtd.h);
this package is its Python binding.  Importing it does not require a GPU;
calls into the library fail loudly if it has not been built.
"""

from ._lib import FdtdError, LIB_PATH, load  # noqa: F401
from .solver import (STORAGE_BITS, STORE_DTYPES, FDTDGrad, Gradient, Problem, codec_roundtrip,  # noqa: F401
                     set_graphs, store_config, timing_enable, timing_read)
from .optimize import DesignLoop  # noqa: F401
