"""Seeded synthetic inputs for the LRBMS online step.

This package builds problem descriptions (grids, permeability and porosity
fields, wells, boundary tags, time step, offline options) and random states.
It holds none of the method's arithmetic: no discretization, no mobility, no
solve.  Both the CPU oracle and the GPU path consume what it produces.
"""
from .problems import (Problem, CONFIGS, make_problem, gaussian_field,
                       face_counts, random_saturation, training_params, smooth_fields,
                       wave_fields, ensemble_caps)

__all__ = ["Problem", "CONFIGS", "make_problem", "gaussian_field", "face_counts",
           "random_saturation", "training_params", "smooth_fields", "wave_fields",
           "ensemble_caps"]
