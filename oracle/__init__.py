"""The oracle: an FP64 CPU reference of the LiDAR simulation path.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import it.  It shares no code with the GPU
library (``paper_2208_10295_amd``) and never imports it.
"""
from .lidar_oracle import *  # noqa: F401,F403
from .lidar_oracle import simulate, first_hit, philox4x32_10, box_muller, beam_directions  # noqa: F401
