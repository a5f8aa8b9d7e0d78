"""Seeded synthetic inputs for the DRK rasterizer.

This package only draws random scenes and cameras.  It holds none of the
rasterizer's arithmetic, so both the HIP library's tests and the CPU oracle can
use it without sharing method code.
"""
from .scenes import (  # noqa: F401
    Camera, Scene, camera_lookat, camera_from_yaw_pitch, intrinsics_hfov,
    draw_angles, draw_quaternions, scene_uniform_box, scene_sphere_shell,
    scene_clusters, config_c1, config_c2, config_c3, config_c4_scenes,
    config_c5, c3_camera_path, random_target,
)
from .meshes import mesh_icosphere, mesh_scene, mesh_torus  # noqa: F401,E402
