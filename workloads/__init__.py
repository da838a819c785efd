"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds input generation only (random fields, PDE discretisation); none of the
sort or solver arithmetic lives here.
"""
from .darcy import (DarcySystem, darcy_from_nodes, darcy_sequence, darcy_system, faces_from_nodes,
                    grf_field, param_matrix, permeability)
from .darcy3d import Darcy3DSystem, darcy3d_sequence, darcy3d_system, grf_field3d

__all__ = ["DarcySystem", "darcy_from_nodes", "darcy_sequence", "darcy_system", "faces_from_nodes",
           "grf_field", "param_matrix", "permeability", "Darcy3DSystem", "darcy3d_sequence", "darcy3d_system",
           "grf_field3d"]
