"""Seeded synthetic inputs (scenes and cameras) shared by the oracle and the GPU path."""
from .scenes import (Scene, Cameras, make_scene, preset_scene, serving_scenes, tiny_camera,
                     full_camera, orbit_cameras, random_cameras, make_cameras, concat_cameras, planes_only, grid_only_scene,
                     maxpool, reachable_mask, mlp_param_count, BLOCK, CHANNELS, MLP_IN,
                     MLP_HIDDEN, MLP_OUT)
