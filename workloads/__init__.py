"""Seeded synthetic workloads shared by the CPU oracle tests and the HIP path.

This package only draws random numbers and does plain ray/box geometry to
synthesise lidar samples.  It holds none of the occupancy method's arithmetic
(no voxel walk, no log-odds, no NDT statistics); both sides of every parity
test receive the same arrays from here.
"""
from .scenes import (  # noqa: F401
    MapParams,
    RayBatch,
    config0,
    config1,
    config2,
    config3,
    config4,
    tunnel_scene,
    label_grid,
    random_rays,
    grid_map,
)
