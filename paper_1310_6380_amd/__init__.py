"""MI355X-native mixed-variational phononic band-structure library (mvpb).

The compute path is the HIP library ``libmvpb.so`` (gfx950), reached through
the C-ABI declared in ``include/mvpb.h`` and the ctypes binding in
:mod:`paper_1310_6380_amd.mvpb`.
"""
from . import mvpb  # noqa: F401
