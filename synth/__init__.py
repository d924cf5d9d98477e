"""Seeded synthetic inputs for narrow-phase contact detection.

This package produces geometry and particle states only: triangle meshes in
their body frame, rigid states (position, unit quaternion, velocity, angular
velocity), packings of bounding spheres and candidate particle pairs from a
bounding-sphere test. It holds none of the narrow-phase arithmetic (no
triangle distances, no rigid-motion evaluation, no time stamps); both the
oracle's tests and the GPU path's tests and benchmarks draw their inputs here.

The paper's own scenes (hopper, staircase, stacks, tower) and its Perlin-noise
particle generator are not available, so the shapes follow its description of
quasi-spherical particles of tens to hundreds of triangles (runtime results
section, the hopper and staircase scenarios) with a uniform radial
perturbation standing in for the noise.
"""

from .meshes import (icosphere, uv_sphere, perturb_radial, mesh_radius,
                     uv_sphere_size)
from .scenes import (random_quaternions, random_unit_vectors, relax_packing, cluster_sizes, cluster_members,
                     rsa_packing, sphere_pairs, Scene, cfg1_scene, cfg2_scene,
                     cfg3_scene, cfg4_scene, cfg5_scene, pair_test_scene)

__all__ = [
    "icosphere", "uv_sphere", "uv_sphere_size", "perturb_radial", "mesh_radius",
    "random_quaternions", "random_unit_vectors", "relax_packing", "rsa_packing",
    "sphere_pairs", "cluster_sizes", "cluster_members", "Scene", "cfg1_scene", "cfg2_scene", "cfg3_scene",
    "cfg4_scene", "cfg5_scene", "pair_test_scene",
]
