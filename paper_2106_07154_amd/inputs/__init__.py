"""Seeded synthetic inputs shared by the GPU path, the oracle and the tests.

This module builds meshes (MPAS-style Voronoi C-grid connectivity and
geometry), fine-region masks and initial states.  It holds none of the time
stepping or right-hand-side arithmetic: region labelling, TRiSK weights,
operators and integrators live separately in the library and in the oracle.
"""
from .mesh import Mesh
from .hexmesh import periodic_hex_mesh
from .cases import (igw_state, igw_parameters, strip_fine_mask, disk_fine_mask,
                    gaussian_bump_state, random_state)

__all__ = ["Mesh", "periodic_hex_mesh", "igw_state", "igw_parameters",
           "strip_fine_mask", "disk_fine_mask", "gaussian_bump_state",
           "random_state"]
