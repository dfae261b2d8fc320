"""Seeded synthetic scene generation (inputs only, shared by the oracle and the GPU path)."""
from .cities import (Scene, tiny_scene, block_scene, district_scene, empty_scene, ground_scene,
                     sealed_box_scene, mirror_scene, config_scene, volumetric_scene, wall_scene, corner_scene)
from .workloads import ScenarioSpec, batch_scenarios, serving_requests, street_points

__all__ = ["Scene", "tiny_scene", "block_scene", "district_scene", "empty_scene", "ground_scene",
           "sealed_box_scene", "mirror_scene", "config_scene", "volumetric_scene", "wall_scene", "corner_scene", "ScenarioSpec", "batch_scenarios",
           "serving_requests", "street_points"]
