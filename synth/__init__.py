"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This package only draws random scenes, cameras and Gaussians. It performs none
of the render path's arithmetic (LOD selection, decoding, projection, binning,
sorting or compositing); both the HIP library and the CPU oracle receive the
arrays it produces and compute everything else on their own.
"""

from .scenes import (  # noqa: F401
    Camera,
    Scene,
    look_at,
    camera_from_yaw_pitch,
    zoomout_trajectory,
    random_views,
    make_scene,
    make_config1,
    make_config2,
    make_config3,
    config3_views,
    perturbed_copy,
    make_config5,
    config5_cameras,
    config5_train_views,
    make_gradcheck_scene,
    random_gaussians,
    tile_aligned_gaussians,
    GAUSS_FIELDS,
)
