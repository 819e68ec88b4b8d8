"""FP64 CPU oracle for MERF deferred volume rendering -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU renderer never uses it.

The arithmetic lives in ``merf_oracle.c`` (plain C, double precision); this
module builds it (``build()``) and marshals numpy arrays through ctypes.
"""
from .oracle import (build, load, OracleScene, render, render_ray, contract, region, map_region,
                     unmap_region, segments, candidates, features, occupied, dequant, encode, mlp,
                     camera_rays, max_threads, RAY_STATS_FIELDS)
