"""Seeded synthetic multilayer stacks.

This module only draws random numbers and packs them into plain stack
descriptions (interface shapes, layer wavenumbers, discretisation sizes,
incident angles).  It holds none of the solver's arithmetic, so the CPU
oracle and the GPU path can both read the same inputs without sharing any
method code.
"""
from .stacks import (Interface, ShapeProblem, Stack, config1, config1_flat, config2, config3, config4, config5,
                     homogeneous, kappa_grid_thetas, small_mixed_stack, small_polygon_stack, small_shape_problem,
                     small_stack)

__all__ = ["Interface", "ShapeProblem", "Stack", "config1", "config1_flat", "config2", "config3", "config4",
           "config5", "homogeneous", "kappa_grid_thetas", "small_mixed_stack", "small_polygon_stack",
           "small_shape_problem", "small_stack"]
