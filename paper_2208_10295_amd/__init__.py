"""MI355X (gfx950) LiDAR simulation after arXiv:2208.10295.

The HIP library ``liblidar.so`` (include/lidar.h) does the work; this package
is its Python binding.  Importing it loads the library and raises if it has
not been built (``python paper_2208_10295_amd/build.py``).
"""
from ._abi import LidarError, NO_LABEL, NO_TRIANGLE, NO_MATERIAL  # noqa: F401
from .lidar import Batch, Context, LidarReturn, LidarSpectralReturn, alloc_outputs, as_u32  # noqa: F401
from .lidar import probe_gather_launcher, probe_stream_launcher  # noqa: F401
