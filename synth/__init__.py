"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package produces *inputs only*: simplex meshes (identified vertex ids plus
unwrapped per-element coordinates), analytic velocity fields as plain
functions of position, and seeded noise / direction vectors.  It contains none
of the method's arithmetic: no basis, no quadrature, no degrees of freedom, no
operator.  Interpolating a field into the discrete space is done separately by
the oracle and by the library.
"""
from .mesh import kuhn_mesh, two_element_mesh, Mesh, graded_nodes, symmetric_graded_nodes
from .fields import (taylor_green_2d, taylor_green_3d, curl_fourier_periodic,
                     curl_fourier_wall, spectral_wall_field, constant_field,
                     shear_field, field_rms)
from .configs import CONFIGS, make_config

__all__ = ["kuhn_mesh", "two_element_mesh", "Mesh", "graded_nodes",
           "symmetric_graded_nodes", "taylor_green_2d", "taylor_green_3d",
           "curl_fourier_periodic", "curl_fourier_wall", "spectral_wall_field",
           "constant_field", "shear_field", "field_rms", "CONFIGS", "make_config"]
