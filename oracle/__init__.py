"""FP64 CPU oracle of the differentiable PSF path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path (the HIP library and its binding)
never imports, calls or links it, and it shares no code with that path.
"""
from .psf import (  # noqa: F401
    OracleProblem, pixel_grid, dft_matrix, focal_field, focal_field_adjoint, opd_map, pupil_field,
    bin_detector, expand_detector, forward, loss_grad, backward, value_and_grad, binned_pixels,
    dither_windows, forward_dithered, backward_dithered, value_and_grad_dithered, intrapixel_grad,
    intrapixel_grad_dithered, kernel_on_focal_grid,
)
