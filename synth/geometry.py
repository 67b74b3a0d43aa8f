"""Input geometry: grids, apertures, Zernike basis, bicubic interpolation matrix.

These arrays are inputs of the optical model, built before it runs, in the
way the paper's listing in Section 3 builds its transmission and basis with
coordinate, circle, combine and Zernike-basis utilities. Nothing here
propagates a field.

Conventions (the paper is silent on them):
* grids are pixel-centred: sample ``i`` of an ``n``-point grid of pitch ``p``
  sits at ``(i - (n - 1) / 2) * p``;
* a pupil array is indexed ``[row, col] = [y, x]``;
* Zernike terms follow Noll's 1976 index order and are normalised to unit
  RMS over the disk of radius D/2, and are zero outside it.
"""
from __future__ import annotations

import math

import numpy as np


def pixel_centres(n: int, pitch: float) -> np.ndarray:
    """Pixel-centred 1-D grid of ``n`` samples with spacing ``pitch`` (FP64)."""
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * pitch


def aperture(n: int, diameter: float, obstruction: float = 0.0, spider_px: float = 0.0,
             supersample: int = 3) -> np.ndarray:
    """Grey transmission of a circular aperture on an ``n``x``n`` pupil grid.

    The clear disk has radius D/2. ``obstruction`` is the diameter of the
    central obstruction as a fraction of D (0 for none). ``spider_px`` > 0
    adds four vanes along +-x and +-y, each ``spider_px`` pupil pixels wide,
    running from the centre to the rim. Edges are anti-aliased by evaluating
    the binary masks on a ``supersample``-times finer grid and averaging each
    block, as the paper's aperture listing (Section 3) does with its
    oversampled circles.
    """
    dx = diameter / n
    s = pixel_centres(n * supersample, dx / supersample)
    X, Y = np.meshgrid(s, s)  # [row=y, col=x]
    R = np.hypot(X, Y)
    t = (R <= diameter / 2.0)
    if obstruction > 0.0:
        t &= R >= obstruction * diameter / 2.0
    if spider_px > 0.0:
        half = 0.5 * spider_px * dx
        t &= ~((np.abs(Y) < half) | (np.abs(X) < half))
    t = t.astype(np.float64).reshape(n, supersample, n, supersample).mean(axis=(1, 3))
    return t


def noll_to_nm(j: int) -> tuple[int, int]:
    """Radial order n and signed azimuthal order m of Noll index ``j`` >= 1.

    Within a radial order, |m| increases; for m != 0 an even ``j`` is the
    cosine term (m > 0) and an odd ``j`` the sine term (m < 0).
    """
    if j < 1:
        raise ValueError("Noll indices start at 1")
    n = 0
    while j > (n + 1) * (n + 2) // 2:
        n += 1
    k = j - n * (n + 1) // 2 - 1  # position inside the radial order, 0..n
    mabs = 2 * ((k + 1) // 2) if n % 2 == 0 else 2 * (k // 2) + 1
    if mabs == 0:
        return n, 0
    return n, (mabs if j % 2 == 0 else -mabs)


def _radial(n: int, m: int, rho: np.ndarray) -> np.ndarray:
    out = np.zeros_like(rho)
    for k in range((n - m) // 2 + 1):
        c = ((-1) ** k * math.factorial(n - k)
             / (math.factorial(k) * math.factorial((n + m) // 2 - k) * math.factorial((n - m) // 2 - k)))
        out += c * rho ** (n - 2 * k)
    return out


def zernike_basis(noll: list[int] | np.ndarray, n: int, diameter: float) -> np.ndarray:
    """Noll Zernike terms on the pixel-centred ``n``x``n`` pupil grid, FP64 [len(noll), n, n]."""
    x = pixel_centres(n, diameter / n)
    X, Y = np.meshgrid(x, x)
    rho = np.hypot(X, Y) / (diameter / 2.0)
    theta = np.arctan2(Y, X)
    inside = rho <= 1.0
    out = np.zeros((len(noll), n, n))
    for i, j in enumerate(noll):
        nn, m = noll_to_nm(int(j))
        r = _radial(nn, abs(m), rho)
        if m == 0:
            z = math.sqrt(nn + 1) * r
        elif m > 0:
            z = math.sqrt(2 * (nn + 1)) * r * np.cos(m * theta)
        else:
            z = math.sqrt(2 * (nn + 1)) * r * np.sin(-m * theta)
        out[i] = np.where(inside, z, 0.0)
    return out


def binary_phase_screen(n: int, rng: np.random.Generator, n_waves: int = 6, max_cycles: float = 6.0) -> np.ndarray:
    """Stand-in for a binary diffractive pupil: phase 0 or pi (a half-wave step) on regions bounded by the
    zero set of a sum of ``n_waves`` random plane waves of up to ``max_cycles`` cycles across the pupil.
    Returned as FP32 radians [n, n]; the real plate's layout is not used."""
    t = (np.arange(n) - (n - 1) / 2.0) / n
    yy, xx = np.meshgrid(t, t, indexing="ij")
    f = np.zeros((n, n))
    for _ in range(n_waves):
        kx, ky = rng.uniform(-max_cycles, max_cycles, size=2)
        f += np.cos(2 * np.pi * (kx * xx + ky * yy) + rng.uniform(0, 2 * np.pi))
    return np.where(f > 0, np.pi, 0.0).astype(np.float32)


def fresnel_defocus_basis(n_pupil: int, diameter: float, focal_length: float) -> np.ndarray:
    """Pupil OPD per metre of detector defocus, -(x^2 + y^2) / (2 f^2), as FP32 [n_pupil, n_pupil].

    Section 1 names the Fresnel regime of a slightly defocused detector: a quadratic phase factor
    before the Fourier transform and another after it. For a detector displaced by delta past the
    focus of a system of focal length f, the factor before the transform is the pupil optical path
    difference -delta (x^2 + y^2) / (2 f^2) (paraxial, delta << f). Appended to the aberration
    basis (rows [N_z, n, n]) with coefficient delta in metres, it models the defocused detector, and
    the gradient with respect to delta is that row's entry of the Zernike gradient. The factor after
    the transform has unit modulus on the focal grid and changes neither |E|^2 nor the gradient, so
    it is not an input; the change of the angular pixel scale by delta / f is neglected at this
    order."""
    if focal_length <= 0:
        raise ValueError("focal_length must be positive")
    x = pixel_centres(n_pupil, diameter / n_pupil)
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    return (-r2 / (2.0 * focal_length ** 2)).astype(np.float32)


def keys_weight(t: np.ndarray, a: float = -0.5) -> np.ndarray:
    """Keys (1981) cubic convolution kernel with parameter ``a``."""
    t = np.abs(t)
    w = np.zeros_like(t)
    near = t <= 1.0
    far = (t > 1.0) & (t < 2.0)
    w[near] = (a + 2) * t[near] ** 3 - (a + 3) * t[near] ** 2 + 1
    w[far] = a * t[far] ** 3 - 5 * a * t[far] ** 2 + 8 * a * t[far] - 4 * a
    return w


def keys_bicubic_matrix(n_pupil: int, n_nodes: int, diameter: float) -> np.ndarray:
    """Separable bicubic interpolation matrix ``B`` [n_pupil, n_nodes] (FP64).

    Nodes are pixel-centred across the diameter (pitch D/n_nodes); pupil
    samples are the pixel centres of the pupil grid. Each row holds the four
    Keys weights (a = -0.5) of the neighbouring nodes, with node indices
    clamped to the edge. A node map ``C`` [n_nodes, n_nodes] becomes the
    pupil map ``B @ C @ B.T``.
    """
    h = diameter / n_nodes
    xn = pixel_centres(n_nodes, h)
    xp = pixel_centres(n_pupil, diameter / n_pupil)
    B = np.zeros((n_pupil, n_nodes))
    t0 = (xp - xn[0]) / h
    j0 = np.floor(t0).astype(int)
    for off in (-1, 0, 1, 2):
        j = j0 + off
        w = keys_weight(t0 - j)
        jc = np.clip(j, 0, n_nodes - 1)
        np.add.at(B, (np.arange(n_pupil), jc), w)
    return B
