"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates inputs*: Kuhn-split grid meshes, boundary and
region masks, material constants, obstacle trajectories and random penalty
sets.  It contains none of the method's arithmetic (no shape operators, no
stiffness, no rotations, no solves), so the CPU oracle and the GPU path can
both draw from it without sharing any code that computes a result.
"""
from .grid import kuhn_grid, kuhn_grid_slit, layer_mask, grid_node_id
from .scenes import (Scene, SphereSchedule, SlitScene, JawSchedule, scene_cube8, scene_slab56,
                     scene_small, scene_irregular, scene_slit, random_penalty_set, slab56_trajectory, lame_mu,
                     POISSON_NU, YOUNG_E, surface_points, top_face_proxy_points, region_tets,
                     LevelSetBodies, slit_levelset_bodies)

__all__ = ["kuhn_grid", "kuhn_grid_slit", "layer_mask", "grid_node_id", "Scene",
           "SphereSchedule", "SlitScene", "JawSchedule", "scene_slit",
           "scene_cube8", "scene_slab56", "scene_small", "scene_irregular", "random_penalty_set", "slab56_trajectory",
           "lame_mu", "POISSON_NU", "YOUNG_E", "surface_points", "top_face_proxy_points",
           "region_tets", "LevelSetBodies", "slit_levelset_bodies"]
