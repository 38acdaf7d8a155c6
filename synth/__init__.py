"""Seeded synthetic inputs for 3D Gabor splatting.

This package only draws random numbers and builds cameras. It holds none of the
method's arithmetic (no projection, no blending), so both the CPU reference and
the GPU path can consume its outputs without sharing any of the method's code.
"""
from .scenes import (  # noqa: F401
    Camera,
    Scene,
    look_at,
    pinhole_camera,
    scene_1k_k2_rgb,
    camera_128,
    scene_1m_k4_sh3,
    camera_1297x840,
    scene_300k_k4_sh3,
    orbit_cameras_64x800,
    serving_scenes,
    serving_requests,
    clustered_scene,
    uniform_scene,
    random_geom,
    random_dl_dimage,
    random_target,
)
