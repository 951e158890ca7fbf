"""Seeded synthetic RGB-D inputs for the alignment and fusion workloads.

This package describes scenes (planes and axis-aligned boxes carrying a solid
Perlin texture), ray-casts them into intensity / inverse-depth frames, adds
sensor noise and holes, and draws camera motions.  It holds none of the
alignment or fusion arithmetic: both the FP64 oracle and the HIP path read
the arrays it produces, and neither is imported here.
"""
from .scene import (Camera, Scene, Frame, Pair, planes3_scene, room_scene,
                    closed_room_scene, render, make_frame, random_motion,
                    compose, invert, relative, pair_c1, pair_c2, walk_c3,
                    batch_c4, pair_warm, keyframe_sequence, camera_640,
                    camera_160, camera_320, camera_1280, to_fp16_grid,
                    track_sequence)

__all__ = [
    "Camera", "Scene", "Frame", "Pair", "planes3_scene", "room_scene",
    "closed_room_scene", "render", "make_frame", "random_motion", "compose",
    "invert", "relative", "pair_c1", "pair_c2", "walk_c3", "batch_c4",
    "pair_warm", "keyframe_sequence", "camera_640", "camera_160",
    "camera_320", "camera_1280", "to_fp16_grid", "track_sequence",
]
