"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle."""
from .generate import (Scene, cached_scene, city_scene, make_scene, path_scene, ring_scene, scaling_scene, sine_field,
                       tiny_scene)

__all__ = ["Scene", "cached_scene", "make_scene", "tiny_scene", "ring_scene", "city_scene", "path_scene", "scaling_scene", "sine_field"]
