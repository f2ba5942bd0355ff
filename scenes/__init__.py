"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle."""
from .generate import Scene, make_scene, tiny_scene, ring_scene, city_scene, path_scene

__all__ = ["Scene", "make_scene", "tiny_scene", "ring_scene", "city_scene", "path_scene"]
