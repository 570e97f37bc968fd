"""MI355X-native programmable-profile incoherent dedispersion and boxcar detection.

The compute path is libdedisp.so (HIP kernels for gfx950 behind the C ABI of
include/dedisp.h); this package only marshals arguments.  Importing it loads
the library and fails loudly if it has not been built.
"""
from . import _lib
from ._lib import DedispError

_lib.lib()  # fail at import time when the HIP library is missing

from .api import Batch, Plan, trial_dms  # noqa: E402
from .stream import StreamDedisperser, StreamSearch  # noqa: E402

__all__ = ["Batch", "Plan", "StreamDedisperser", "StreamSearch", "trial_dms", "DedispError"]
