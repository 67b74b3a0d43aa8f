"""Host-side builders of optical inputs that reduce to the library's pupil terms.

Fresnel defocus (Section 1: a detector slightly out of focus adds a
quadratic phase factor before the Fourier transform and another after it).
For a detector displaced by delta along the beam, past the focus of a
system of focal length f, the factor before the transform is the pupil
optical path difference -delta (x^2 + y^2) / (2 f^2) (paraxial, delta << f);
``fresnel_defocus_basis`` returns that map per metre of delta, so it enters
the library as one more row of the aberration basis with coefficient delta,
and its gradient comes back in the Zernike-gradient slot of that row. The
factor after the transform has unit modulus on the focal grid: it changes
neither |E|^2 nor the adjoint seed's contribution to the pupil gradient, so
nothing is applied for it. The detector's angular pixel scale changes by
delta / f, which is neglected at this order.

Static phase screens (Section 3: the paper's system carries a binary phase
plate after the Zernike aperture) go through ``PsfPlan.set_phase_screen``.
"""
from __future__ import annotations

import numpy as np


def pupil_coordinates(n_pupil: int, diameter: float) -> np.ndarray:
    """Pixel-centred pupil sample coordinates in metres, (i - (n-1)/2) * diameter / n (the library's grid)."""
    return (np.arange(n_pupil) - (n_pupil - 1) / 2.0) * (diameter / n_pupil)


def fresnel_defocus_basis(n_pupil: int, diameter: float, focal_length: float) -> np.ndarray:
    """Pupil OPD per metre of detector defocus, -(x^2 + y^2) / (2 f^2), as FP32 [n_pupil, n_pupil].

    Append it to the Zernike basis (rows [N_z, n, n]) with coefficient delta (metres; positive past the
    focus) to model a slightly defocused detector; the gradient of the loss with respect to delta is
    the gradient entry of that row."""
    if focal_length <= 0:
        raise ValueError("focal_length must be positive")
    x = pupil_coordinates(n_pupil, diameter)
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    return (-r2 / (2.0 * focal_length ** 2)).astype(np.float32)
