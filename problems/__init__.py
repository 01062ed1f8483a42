"""Seeded synthetic inputs shared by the HIP path, its tests and the CPU oracle.

This package holds only input generation (coefficient fields, loads, boundary
data, sensors, random directions).  It contains none of the method's
arithmetic: no stencil, no elimination, no interface system.
"""
from .synthetic import (Problem, fourier_field, make_config, config_names,
                        sensor_nodes, fd_directions, box_boundary_values, perturbed_kappa)

__all__ = ["Problem", "fourier_field", "make_config", "config_names",
           "sensor_nodes", "fd_directions", "box_boundary_values", "perturbed_kappa"]
