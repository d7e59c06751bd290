"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This package holds no arithmetic of the solver: it only samples media m(x),
potentials V(x), incident plane waves u_I(x) = exp(i omega dhat . x), delta
sources, general-domain masks with their cavity media and Gaussian sketch
matrices, and random test vectors on the grid, from fixed seeds.  Both the oracle and the HIP path consume the
arrays it returns; neither side's solver code lives here.

Grid convention (the paper's uniform grid with step h, Section 2.1, read as
cell-centred): h = 1/n, x_i = (i + 1/2) h for i in {0..n-1}^d, linear index
l = i1 + n*i2 (+ n^2*i3), i1 fastest.
"""
from .media import (grid_coords, medium_single_bump, medium_bumps, medium_disks,
                    plane_waves, directions_2d, directions_fibonacci,
                    random_rotation, workload, WORKLOADS, random_complex,
                    serving_requests, potential_gaussian, potential_ball, delta_source,
                    cavity_rho, domain_mask, medium_cavity, sketch_matrix)

__all__ = ["grid_coords", "medium_single_bump", "medium_bumps", "medium_disks",
           "plane_waves", "directions_2d", "directions_fibonacci",
           "random_rotation", "workload", "WORKLOADS", "random_complex",
           "serving_requests", "potential_gaussian", "potential_ball", "delta_source",
           "cavity_rho", "domain_mask", "medium_cavity", "sketch_matrix"]
