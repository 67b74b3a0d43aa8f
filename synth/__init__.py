"""Seeded synthetic inputs for the differentiable PSF path.

This package builds the *inputs* of the forward model and nothing else:
pupil grids, aperture transmission, the Zernike basis, the bicubic
map-to-pupil interpolation matrix, random parameter draws, dithers and the
workload shapes. It contains none of the propagation, binning, flat-field,
loss or gradient arithmetic; those live, independently, in the HIP library
and in the FP64 oracle. Both sides read their inputs from here.
"""
from .geometry import (pixel_centres, aperture, noll_to_nm, zernike_basis, keys_bicubic_matrix,  # noqa: F401
                       binary_phase_screen, fresnel_defocus_basis)
from .configs import (Problem, Workload, make_problem, make_workload, make_c4_workloads, standin_image,  # noqa: F401
                      intrapixel_kernel, CONFIG_NAMES, DEFAULT_DIAMETER, DitheredWorkload, make_dithered_workload,
                      dithered_standin_image)
