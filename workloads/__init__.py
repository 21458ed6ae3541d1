"""Seeded synthetic inputs for the Schur-interface elasticity solver.

This package only *describes* problems: mesh sizes, subdomain cuts, the
Poisson ratio, the clamped faces, element moduli E_e and the nodal load
vector f.  It contains none of the method's arithmetic (no element
matrices, no assembly, no solves), so both the CPU oracle and the GPU path
may use it to build the same inputs.
"""
from .gen import (  # noqa: F401
    Problem,
    CLAMP_X0,
    gaussian_random_field,
    simp_moduli,
    cantilever2d,
    cantilever3d,
    cantilever2d_uniform_64x32,
    cantilever2d_simp_512x256,
    cantilever3d_simp,
    cantilever3d_simp_128x64x64,
    to_sequence_2d,
    to_sequence_3d,
    simp_sequence_3d,
    cnn_initial_weights,
    batch_uneven_problem,
    even_cuts,
)
