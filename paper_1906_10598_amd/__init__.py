"""MI355X-native phase-tracking fit (arXiv:1906.10598): HIP kernels behind a C ABI.

``phasetrack`` is the ctypes binding of ``libphasetrack.so``; the C header is
``include/phasetrack.h``.
"""
from . import phasetrack  # noqa: F401
from .phasetrack import Context  # noqa: F401
