"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the benchmark.

This module only draws random numbers and lays out triangles, weights and label masks.
It holds none of the method's arithmetic (no froxel overlap, no interleave, no convolution),
so the oracle and the HIP path can both consume its output without sharing code.
"""
from .scenes import (  # noqa: F401
    box_scene, city_scene, he_weights, label_mask_bits, viewpoints, CONFIGS, config,
    net_layers, scene_for, unet_params,
)
