"""Glue between the seeded inputs and the FP64 oracle (test-side only)."""
import numpy as np

from oracle import OracleProblem


def oracle_problem(w):
    P = w.problem
    return OracleProblem.from_arrays(P.n_pupil, P.n_focal, P.oversample, P.diameter, P.focal_pixel,
                                     P.wavelengths, P.weights, w.transmission, w.zbasis,
                                     w.map_basis, w.intrapixel)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    a = a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)
    b = b.astype(np.complex128 if np.iscomplexobj(b) else np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))
