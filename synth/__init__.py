"""Seeded synthetic inputs shared by the HIP library's tests and the oracle.

This package prepares inputs only (graphs, sampling sets, sampled data); it
contains none of the solvers' arithmetic.
"""
from .graphs import knn_indices, knn_laplacian, laplacian_lmax, low_eigvecs  # noqa: F401
from .configs import (Problem, cfg1_tiny, cfg2_face, cfg3_video, cfg5_batch,  # noqa: F401
                      small_problem, make_problem, round_count, grid_coords,
                      circle_coords, helix_coords, cluster_digits, digits_points)
