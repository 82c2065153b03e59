"""Seeded synthetic inputs shared by the GPU path's tests and benchmark and the oracle."""
from .scenes import (Scene, Sensor, Pose, Instance, Mesh, Actor, config1, config2, config3, config4, config5,
                     dynamic_config, car_mesh, pedestrian_mesh, pedestrian_pose_vertices,
                     elev_table, quat_from_ypr, urban_small, urban_large, N_BINS, LAMBDA0_NM, DLAMBDA_NM)
