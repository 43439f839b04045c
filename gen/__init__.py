"""Seeded synthetic finite-element inputs for the patch-relaxation path."""
from .fem import (Problem, q1_poisson_2d, taylor_hood_stokes_2d, nedelec_hex,
                  q2_hex_diffusion, uneven_stokes_batch, rhs, lognormal_field,
                  nedelec_regions, qp_diffusion_2d, tensor_interpolation, tensor_node_coords,
                  qp_hex_diffusion)
from .configs import make_config, CONFIG_NAMES

__all__ = ["Problem", "q1_poisson_2d", "taylor_hood_stokes_2d", "nedelec_hex",
           "q2_hex_diffusion", "uneven_stokes_batch", "rhs", "make_config",
           "CONFIG_NAMES", "lognormal_field", "nedelec_regions", "qp_diffusion_2d",
           "tensor_interpolation", "tensor_node_coords", "qp_hex_diffusion"]
