"""MI355X-native NLOS reconstruction hot path: photon binning, f-k migration and
radial phasor-field RSD as hand-written HIP kernels for gfx950 behind the C ABI
of include/nlos.h.  ``nlos`` is the ctypes binding (same names as the C calls);
``runtime`` adds tensor-level helpers and the serving loop lives in ``serve``.
"""
from . import nlos  # noqa: F401
