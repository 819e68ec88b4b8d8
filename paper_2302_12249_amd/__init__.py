"""MERF deferred volume rendering on MI355X (gfx950).

The renderer is the HIP library ``libmerf_hip.so`` behind the C ABI in
``include/merf.h``; :mod:`paper_2302_12249_amd.merf` is its ctypes binding.
"""
from . import merf  # noqa: F401
