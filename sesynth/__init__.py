"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds input recipes only (meshes, bathymetry, forcing, initial
fields); it contains none of the scheme's arithmetic.
"""
from .meshes import BASE_SEED, rng, planar_grid, latlon_grid, grid_triangles, tiny_mesh  # noqa: F401
from .configs import (make_config, basin_c1, channel_c2, latlon_c3, batch_c4, vertex_subset,  # noqa: F401
                      adjoint_c5, torus, equilateral_torus, random_case, layers, column_forcing,
                      G, THETA,
                      OMEGA)
