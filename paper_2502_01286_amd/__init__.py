"""Segmented NCC template matching on MI355X (gfx950).

The work is done by ``libsncc.so`` (HIP kernels behind the C-ABI declared in
``include/sncc.h``); this package is its thin Python binding.  Importing it
raises ImportError when the library has not been built
(``python paper_2502_01286_amd/build.py``).
"""

from ._native import *  # noqa: F401,F403
from ._native import (  # noqa: F401
    Batch,
    SEGMENT_DTYPE,
    SnccError,
    decode_matches,
    decode_matches64,
    decode_hits,
    header_functions,
    lib,
)
