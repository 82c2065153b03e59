"""Seeded synthetic inputs shared by the GPU path's tests and benchmark and the oracle."""
from .scenes import (Scene, Sensor, Pose, Instance, Mesh, Actor, small_16ch, urban_64ch, urban_sequence_128ch, batch_256, calibration_20mat,
                     dynamic_actors, car_mesh, pedestrian_mesh, pedestrian_pose_vertices,
                     elev_table, quat_from_ypr, urban_small, urban_large, N_BINS, LAMBDA0_NM, DLAMBDA_NM)
