"""Seeded synthetic inputs for the graph Ginzburg-Landau solves.

This package only builds inputs: point clouds, images, patch features,
k-nearest-neighbour graphs with self-tuning Gaussian weights (stored in CSR),
label masks and initial label fields.  It contains none of the solver's
arithmetic (no degree normalisation, no Laplacian, no sweep, no energy), so
the CPU oracle and the HIP path can both consume its output without sharing
any method code.
"""

from .graphs import (  # noqa: F401
    Graph,
    gaussian_mixture,
    knn_bruteforce,
    window_knn,
    self_tuning_graph,
    rectangles_image,
    textured_regions_image,
    patch_features,
    random_labels,
    initial_u,
    tiny_graph,
    zorder,
)
from .configs import Problem, make_problem, CONFIG_NAMES  # noqa: F401
