"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the CPU oracle.

This package generates *inputs only*: scan geometry (source orbits and detector
frames), random-ellipsoid phantoms and their exact line integrals, Poisson noise
and plain random arrays.  It contains none of the reconstruction method's
arithmetic (no weighting, Radon transform, filtering or backprojection), so the
oracle and the GPU path can both draw from it without sharing method code.
"""
from .geometry import (Grid, Views, radon_bins, circle_orbit, sinusoid_orbit,
                       circle_arc_orbit, circle_line_orbit, random_nn_orbit,
                       config_geometry, paper_geometry, CONFIGS, c4_scans, C4_MIX)
from .phantom import (MU_WATER_PER_MM, Ellipsoids, random_ellipsoids, ball, voxelize, voxelize_torch, project_ellipsoids,
                      gaussian_blobs, project_gaussian_blobs, add_poisson_noise, rand_array)

__all__ = ["Grid", "Views", "radon_bins", "circle_orbit", "sinusoid_orbit",
           "circle_arc_orbit", "circle_line_orbit", "random_nn_orbit",
           "config_geometry", "paper_geometry", "CONFIGS", "c4_scans", "C4_MIX", "Ellipsoids", "random_ellipsoids", "ball",
           "gaussian_blobs", "project_gaussian_blobs",
           "voxelize", "voxelize_torch", "project_ellipsoids", "add_poisson_noise", "rand_array"]
