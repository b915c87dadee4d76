"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds input generation only: cameras and the rays they cast,
random grids and network weights, the random sphere scene, per-ray jitter and
target colours.  It contains none of the rendering method's arithmetic
(no clipping, sampling, interpolation, activation, compositing or gradients),
so that the CPU oracle and the GPU path can both draw identical inputs from it
without sharing any of the computation under test.

All arrays are numpy; ray geometry and grid values are float32 because that is
what both implementations consume.
"""

from .scenes import (  # noqa: F401
    look_at_c2w,
    pixel_rays,
    cube_vertex_cameras,
    hemisphere_cameras,
    draw_pixels_without_replacement,
    draw_pixels_with_replacement,
    random_spheres,
    sphere_field,
    coarse_raw_from_spheres,
    xavier_uniform_mlp,
    image_rays,
    binary_image,
    tiny_config,
    full_config,
    full_scene,
    stress_config,
    Problem,
    RayBatch,
    Spheres,
    BOX_MIN,
    BOX_MAX,
    FULL_N,
    FULL_COARSE_N,
    FULL_ALPHA_INIT,
    FULL_TAU,
    STRESS_N,
    STRESS_MAX_SAMPLES,
    STRESS_ALPHA_INIT,
)
