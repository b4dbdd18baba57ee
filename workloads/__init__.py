"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package holds geometry (triangle meshes), material / excitation records and
seeded random vectors only.  It contains none of the method's arithmetic: no
Green's functions, no basis functions, no grids, no quadrature.  Both the CPU
oracle (``oracle/``) and the HIP library's tests and benchmark draw their inputs
from here, so that the two sides see identical meshes and vectors while sharing
no computation.
"""
from .meshes import (icosphere, geodesic_sphere, box_mesh, cube_array, ellipsoid,
                     mesh_stats, voxel_mesh, split_ring)
from .configs import (Problem, ObjectSpec, PlaneWave, sphere_cfg, bar_cfg, bar_small_cfg,
                      cube_array_cfg, batching_meshes, serving_trace, random_vector,
                      C0_NOMINAL)

__all__ = [
    "icosphere", "geodesic_sphere", "box_mesh", "cube_array", "ellipsoid", "mesh_stats", "voxel_mesh",
    "split_ring",
    "Problem", "ObjectSpec", "PlaneWave", "sphere_cfg", "bar_cfg", "bar_small_cfg",
    "cube_array_cfg", "batching_meshes", "serving_trace", "random_vector", "C0_NOMINAL",
]
