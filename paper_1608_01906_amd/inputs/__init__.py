"""Seeded synthetic inputs (meshes, parameters, initial fields).

Shared by the oracle-side tests and the device path; holds none of the
method's arithmetic.
"""
from .mesh import box_mesh, grid_mesh_2d, grid_mesh_3d, pipe_mesh_3d, splitmix64, uniform01, mesh_summary  # noqa: F401
from .mesh_files import read_gmsh, write_gmsh  # noqa: F401
from .workloads import (Phys, Instance, Workload, WORKLOADS, droplet2d, droplet3d,  # noqa: F401
                        channel2d, rt2d, ensemble2d, translate2d, droplet_instance, channel_profile,
                        pipe3d, pipe_study3d, pipe_instance, pipe_profile, box_droplet, DT_RUN)
