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
    config1_scene,
    config1_camera,
    config2_scene,
    config2_camera,
    config4_scene,
    config4_cameras,
    config5_scenes,
    config5_requests,
    clustered_scene,
    uniform_scene,
    random_geom,
    random_dl_dimage,
    random_target,
)
