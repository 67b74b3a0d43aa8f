"""Plain FP64 direct-DFT model of the PSF path and its analytic gradient.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU baseline; never by the product path.

What it computes follows the paper (Desdoigts et al., "Differentiable optics
with dLux I", arXiv 2406.08703):

* Section 3, aperture listing: a basis optic whose optical path difference
  is a linear combination of Zernike terms over a grey transmission, with
  the field normalised to unit power;
* Section 3, propagation paragraph: Fraunhofer propagation to the focal
  plane by a two-sided matrix Fourier transform, one product per side;
  summed incoherently over wavelengths and stars; pixel response applied
  by multiplication;
* Section 4: a per-pixel Poisson log-likelihood plus a chi-squared prior on
  the pixel response, differentiated with respect to star positions,
  fluxes, Zernike coefficients and every pixel-response value.

The MFT is a direct DFT evaluated at arbitrary output coordinates, so the
oracle is that definition written out with explicit DFT matrices (no FFT),
one PSF at a time, in FP64. Where the paper is silent this module reads it
as follows: the pupil is normalised to unit power and the field scaled by
dx du / lambda (Parseval on a full-period grid); grids are pixel-centred;
the kernel is exp(-2 pi i x u / lambda); binning sums the Q x Q focal
samples of a pixel, weighted by the intra-pixel kernel; the prior is the
Gaussian (F - mu)^2 / (2 sigma^2); the chi-squared data term is
(m - d)^2 / (2 max(d, 1)); the bicubic map's interpolation matrix (an input)
uses Keys' kernel with a = -1/2.

Pins (tests/test_oracle_pins.py): brute-force DFT, FFT equivalence,
Parseval, Airy and annular-Airy closed forms, shift theorem, piston and
even-mode invariances, adjoint dot product, Euler identity for the flux
gradient, library log-pmf/log-pdf for the loss, matrix-form binning, and
central finite differences of every gradient block.
The integer-dither form (``forward_dithered`` / ``backward_dithered``,
Section 3: one PSF computation on an enlarged plane, each frame a window of
it) is pinned to the per-frame form with the dithers folded into the star
positions, by the shift theorem on the focal grid.
The static phase screen (Section 3's fixed phase optic) is pinned by a
constant screen acting as a global phase, by its equivalence with an OPD
at one wavelength, by the sign flip a half-wave plate gives its region
(linearity of the transform) and by finite differences; the Fresnel
defocus basis row is pinned by angular-spectrum propagation of the focal
field on a full-period grid.
Parity unpinned beyond finite differences: the bicubic map term and the
chi-squared data term (definitions, not results).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclass
class OracleProblem:
    """Static inputs of one problem, promoted to FP64."""
    n_pupil: int
    n_focal: int
    oversample: int
    diameter: float
    focal_pixel: float
    wavelengths: np.ndarray
    weights: np.ndarray
    transmission: np.ndarray          # [Ni, Ni]
    zbasis: np.ndarray                # [Nz, Ni, Ni]
    map_basis: np.ndarray | None = None   # [Ni, n_map]
    intrapixel: np.ndarray | None = None  # [Q, Q] shared by every pixel, or [Nd, Nd, Q, Q] per pixel
    phase_screen: np.ndarray | None = None  # [Ni, Ni] static achromatic phase, radians

    @staticmethod
    def from_arrays(n_pupil, n_focal, oversample, diameter, focal_pixel, wavelengths, weights,
                    transmission, zbasis, map_basis=None, intrapixel=None, phase_screen=None) -> "OracleProblem":
        f64 = lambda a: None if a is None else np.asarray(a, dtype=np.float64)
        return OracleProblem(int(n_pupil), int(n_focal), int(oversample), float(diameter), float(focal_pixel),
                             f64(wavelengths), f64(weights), f64(transmission), f64(zbasis),
                             f64(map_basis), f64(intrapixel), f64(phase_screen))

    @property
    def n_det(self) -> int:
        return self.n_focal // self.oversample

    @property
    def dx(self) -> float:
        return self.diameter / self.n_pupil


def pixel_grid(n: int, pitch: float) -> np.ndarray:
    """Pixel-centred sample coordinates ``(i - (n-1)/2) * pitch``."""
    return (np.arange(n) - (n - 1) / 2.0) * pitch


def dft_matrix(x: np.ndarray, u: np.ndarray, lam: float) -> np.ndarray:
    """M[l, n] = exp(-2 pi i x_n u_l / lambda): one side of the two-sided MFT (Section 3)."""
    return np.exp(-1j * TWO_PI * np.outer(u, x) / lam)


def focal_field(P, x, y, u, v, lam, scale):
    """E[k, l] = scale * sum_{m,n} P[m, n] exp(-2 pi i (y_m v_k + x_n u_l) / lambda).

    The two matrix products of Section 3's propagation paragraph:
    ``E = scale * My @ P @ Mx.T``. ``scale`` is dx*du/lambda for the model.
    """
    return scale * (dft_matrix(y, v, lam) @ P @ dft_matrix(x, u, lam).T)


def focal_field_adjoint(Y, x, y, u, v, lam, scale):
    """Adjoint of ``focal_field`` in P: ``scale * My^H @ Y @ conj(Mx)``."""
    return scale * (dft_matrix(y, v, lam).conj().T @ Y @ dft_matrix(x, u, lam).conj())


def opd_map(zbasis, coeffs, map_basis=None, phase_map=None):
    """OPD = sum_j c_j Z_j (Section 3, basis optic), plus the bicubic map B C B^T if given."""
    o = np.tensordot(np.asarray(coeffs, np.float64), zbasis, axes=1)
    if map_basis is not None and phase_map is not None:
        o = o + map_basis @ np.asarray(phase_map, np.float64) @ map_basis.T
    return o


def pupil_field(transmission, opd, x, y, alpha, beta, lam, screen=None):
    """Unit-power pupil field A/sqrt(sum A^2) * exp(i 2 pi/lambda (OPD + x alpha + y beta)) [* exp(i screen)].

    The source at angular offset (alpha, beta) tilts the incoming wavefront.
    ``screen`` is a static phase optic in radians, the same at every
    wavelength (Section 3's system applies such a layer, a binary phase
    plate, after the Zernike aperture).
    """
    amp = transmission / np.sqrt(np.sum(transmission ** 2))
    phase = (TWO_PI / lam) * (opd + x[None, :] * alpha + y[:, None] * beta)
    if screen is not None:
        phase = phase + screen
    return amp * np.exp(1j * phase)


def kernel_on_focal_grid(K, n, Q):
    """The intra-pixel kernel laid on the focal grid: K[a, b] at sample (Qp + a, Qq + b) of every pixel
    (p, q) for a shared kernel [Q, Q], or K[p, q, a, b] for one kernel per pixel [n, n, Q, Q]."""
    K = np.asarray(K, np.float64)
    if K.ndim == 2:
        return np.tile(K, (n, n))
    return K.transpose(0, 2, 1, 3).reshape(n * Q, n * Q)


def bin_detector(I, Q, K=None):
    """B[p, q] = sum_{a,b<Q} K[a, b] I[Qp+a, Qq+b] (K = 1 if None; K[p, q, a, b] if per pixel)."""
    n = I.shape[-1] // Q
    if K is not None:
        I = I * kernel_on_focal_grid(K, n, Q)
    return I.reshape(n, Q, n, Q).sum(axis=(1, 3))


def expand_detector(G, Q, K=None):
    """Adjoint of ``bin_detector``: G[k, l] = K[k%Q, l%Q] * g[k//Q, l//Q] (per pixel: K[k//Q, l//Q, ...])."""
    out = np.kron(G, np.ones((Q, Q)))
    if K is not None:
        out = out * kernel_on_focal_grid(K, G.shape[0], Q)
    return out


def _grids(prob: OracleProblem):
    x = pixel_grid(prob.n_pupil, prob.dx)
    u = pixel_grid(prob.n_focal, prob.focal_pixel)
    return x, u


def _psf_field(prob, opd, x, u, alpha, beta, lam):
    P = pupil_field(prob.transmission, opd, x, x, alpha, beta, lam, prob.phase_screen)
    c = prob.dx * prob.focal_pixel / lam
    return P, focal_field(P, x, x, u, u, lam, c), c


def forward(prob: OracleProblem, coeffs, phase_map, sources, flat):
    """Binned image B [F, Nd, Nd] and model m = flat * B (Section 3).

    ``sources`` is [F, S, 3]: per frame and star the angular position
    (alpha, beta) in radians -- dither included -- and the photon count.
    I_f = sum_s sum_lambda w_lambda * phi_s * |E|^2, then Q x Q binning with
    the intra-pixel kernel, then the pixel response.
    """
    sources = np.asarray(sources, np.float64)
    flat = np.asarray(flat, np.float64)
    x, u = _grids(prob)
    opd = opd_map(prob.zbasis, coeffs, prob.map_basis, phase_map)
    F, S = sources.shape[:2]
    No = prob.n_focal
    binned = np.zeros((F, prob.n_det, prob.n_det))
    for f in range(F):
        I = np.zeros((No, No))
        for s in range(S):
            a, b, phi = sources[f, s]
            for lam, w in zip(prob.wavelengths, prob.weights):
                _, E, _ = _psf_field(prob, opd, x, u, a, b, lam)
                I += w * phi * np.abs(E) ** 2
        binned[f] = bin_detector(I, prob.oversample, prob.intrapixel)
    return binned, flat[None] * binned


def loss_grad(model, binned, data, flat, kind="poisson", prior_mu=1.0, prior_sigma=0.1):
    """Loss, residual r = dL/dm and flat-field gradient (Section 4).

    Poisson: l = m - d ln m (the ln d! constant dropped).
    chi2:    l = (m - d)^2 / (2 max(d, 1)).
    Prior:   sum_p (F_p - mu)^2 / (2 sigma^2).
    dL/dF_p = sum_f r_fp B_fp + (F_p - mu) / sigma^2.
    Returns (L, r, dL/dF, domain_flag); m <= 0 is clamped to 1e-30 and flagged.
    """
    m = np.asarray(model, np.float64)
    d = np.asarray(data, np.float64)
    Fl = np.asarray(flat, np.float64)
    bad = bool(np.any(m <= 0.0))
    m = np.maximum(m, 1e-30)
    if kind == "poisson":
        ell = m - d * np.log(m)
        r = 1.0 - d / m
    elif kind == "chi2":
        wgt = np.maximum(d, 1.0)
        ell = 0.5 * (m - d) ** 2 / wgt
        r = (m - d) / wgt
    else:
        raise ValueError(kind)
    L = float(np.sum(ell) + np.sum((Fl - prior_mu) ** 2) / (2.0 * prior_sigma ** 2))
    gF = np.sum(r * np.asarray(binned, np.float64), axis=0) + (Fl - prior_mu) / prior_sigma ** 2
    return L, r, gF, bad


def backward(prob: OracleProblem, coeffs, phase_map, sources, flat, r):
    """Gradients of L through the optics given r = dL/dm [F, Nd, Nd].

    Per (frame, star, wavelength), recomputing E:
      G = K * expand(F * r)        (dL/dI)
      Y = w phi G E                (dL/dE*)
      W = adjoint MFT of Y
      g = 2 Im(conj(P) W)          (dL/dphase)
    and dL/dc_j = sum (2 pi/lambda) Z_j g; dL/dalpha = sum (2 pi/lambda) x g;
    dL/dbeta likewise with y; dL/dphi = sum_lambda w sum G |E|^2.
    Returns (grad_coeffs [Nz], grad_map [n_map, n_map] or None, grad_sources [F, S, 3]).
    """
    sources = np.asarray(sources, np.float64)
    flat = np.asarray(flat, np.float64)
    r = np.asarray(r, np.float64)
    x, u = _grids(prob)
    opd = opd_map(prob.zbasis, coeffs, prob.map_basis, phase_map)
    F, S = sources.shape[:2]
    g_opd = np.zeros((prob.n_pupil, prob.n_pupil))
    g_src = np.zeros((F, S, 3))
    for f in range(F):
        G = expand_detector(flat * r[f], prob.oversample, prob.intrapixel)
        for s in range(S):
            a, b, phi = sources[f, s]
            for lam, w in zip(prob.wavelengths, prob.weights):
                P, E, c = _psf_field(prob, opd, x, u, a, b, lam)
                Y = w * phi * G * E
                W = focal_field_adjoint(Y, x, x, u, u, lam, c)
                g = 2.0 * np.imag(np.conj(P) * W) * (TWO_PI / lam)
                g_opd += g
                g_src[f, s, 0] += np.sum(g * x[None, :])
                g_src[f, s, 1] += np.sum(g * x[:, None])
                g_src[f, s, 2] += w * np.sum(G * np.abs(E) ** 2)
    g_c = np.tensordot(prob.zbasis, g_opd, axes=([1, 2], [0, 1]))
    g_map = None
    if prob.map_basis is not None and phase_map is not None:
        g_map = prob.map_basis.T @ g_opd @ prob.map_basis
    return g_c, g_map, g_src


def intrapixel_grad(prob: OracleProblem, coeffs, phase_map, sources, flat, r):
    """dL/dK of the intra-pixel kernel (Section 6: recovering intra-pixel sensitivity).

    B_f[p] = sum_ab K[a, b] I_f[Qp + (a, b)] is linear in K, so
    dL/dK[a, b] = sum_f sum_p flat[p] r_f[p] I_f[Qp + (a, b)], with I_f the
    unbinned focal intensity sum_s sum_lambda w phi |E|^2 (recomputed here):
    [Q, Q] for a shared kernel. With one kernel per pixel (prob.intrapixel
    [Nd, Nd, Q, Q]) the sum over p is dropped: [Nd, Nd, Q, Q].
    """
    sources = np.asarray(sources, np.float64)
    flat = np.asarray(flat, np.float64)
    r = np.asarray(r, np.float64)
    x, u = _grids(prob)
    opd = opd_map(prob.zbasis, coeffs, prob.map_basis, phase_map)
    F, S = sources.shape[:2]
    Q = prob.oversample
    No = prob.n_focal
    per_pixel = prob.intrapixel is not None and np.ndim(prob.intrapixel) == 4
    n = prob.n_det
    g = np.zeros((n, n, Q, Q) if per_pixel else (Q, Q))
    for f in range(F):
        I = np.zeros((No, No))
        for s in range(S):
            a, b, phi = sources[f, s]
            for lam, w in zip(prob.wavelengths, prob.weights):
                _, E, _ = _psf_field(prob, opd, x, u, a, b, lam)
                I += w * phi * np.abs(E) ** 2
        h = flat * r[f]
        v = (np.kron(h, np.ones((Q, Q))) * I).reshape(n, Q, n, Q)
        g += v.transpose(0, 2, 1, 3) if per_pixel else v.sum(axis=(0, 2))
    return g


def value_and_grad(prob, coeffs, phase_map, sources, flat, data, kind="poisson", prior_mu=1.0, prior_sigma=0.1):
    """Forward, loss and all gradients in one call (a convenience for tests and the baseline)."""
    B, m = forward(prob, coeffs, phase_map, sources, flat)
    L, r, gF, bad = loss_grad(m, B, data, flat, kind, prior_mu, prior_sigma)
    g_c, g_map, g_src = backward(prob, coeffs, phase_map, sources, flat, r)
    return dict(binned=B, model=m, loss=L, r=r, grad_flat=gF, grad_coeffs=g_c, grad_map=g_map,
                grad_sources=g_src, domain=bad)


def binned_pixels(prob: OracleProblem, coeffs, phase_map, sources, frame, pixels):
    """B_f at selected detector pixels [(p, q), ...], evaluating E only on their Q x Q samples.

    The same definition as ``forward`` with the DFT taken at the needed
    output coordinates only, for spot checks at sizes where the full oracle
    is too slow.
    """
    sources = np.asarray(sources, np.float64)
    x, u = _grids(prob)
    opd = opd_map(prob.zbasis, coeffs, prob.map_basis, phase_map)
    Q = prob.oversample
    Kf = kernel_on_focal_grid(prob.intrapixel if prob.intrapixel is not None else np.ones((Q, Q)), prob.n_det, Q)
    out = np.zeros(len(pixels))
    for s in range(sources.shape[1]):
        a, b, phi = sources[frame, s]
        for lam, w in zip(prob.wavelengths, prob.weights):
            P = pupil_field(prob.transmission, opd, x, x, a, b, lam, prob.phase_screen)
            for i, (p, q) in enumerate(pixels):
                rows = u[Q * p:Q * p + Q]
                cols = u[Q * q:Q * q + Q]
                E = focal_field(P, x, x, cols, rows, lam, prob.dx * prob.focal_pixel / lam)
                out[i] += w * phi * np.sum(Kf[Q * p:Q * p + Q, Q * q:Q * q + Q] * np.abs(E) ** 2)
    return out


def dither_windows(dithers, margin):
    """Top-left corner (row, col) of each frame's window in the enlarged plane.

    ``dithers`` [F, 2] are integer detector-pixel offsets (dx, dy) of the scene
    in frame f; the enlarged plane has ``margin`` extra pixels on every side,
    so detector pixel p of frame f is enlarged-plane pixel p + margin - d_f.
    """
    d = np.asarray(dithers, np.int64)
    if np.any(np.abs(d) > margin):
        raise ValueError("dither larger than the margin")
    return np.stack([margin - d[:, 1], margin - d[:, 0]], axis=1)


def forward_dithered(prob_big: OracleProblem, coeffs, phase_map, sources, flat, dithers, margin):
    """Integer-dithered frames from one enlarged plane (Section 3).

    Every (star, wavelength) PSF is computed once on the enlarged focal grid
    of ``prob_big`` (N_det + 2 margin detector pixels, same pitch), binned
    there, and frame f's binned image is its window at ``dither_windows``.
    ``sources`` is [S, 3] (shared by all frames). Returns (binned, model)
    [F, Nd, Nd].
    """
    flat = np.asarray(flat, np.float64)
    nd = flat.shape[0]
    if prob_big.n_det != nd + 2 * margin:
        raise ValueError("enlarged plane size")
    big, _ = forward(prob_big, coeffs, phase_map, np.asarray(sources, np.float64)[None], np.ones((prob_big.n_det,) * 2))
    win = dither_windows(dithers, margin)
    binned = np.stack([big[0, r:r + nd, c:c + nd] for r, c in win])
    return binned, flat[None] * binned


def backward_dithered(prob_big: OracleProblem, coeffs, phase_map, sources, flat, r, dithers, margin):
    """Adjoint of ``forward_dithered``: dL/dB_big = sum_f (flat * r_f) placed in frame f's window,
    then the adjoint of one enlarged frame with unit pixel response.
    Returns (grad_coeffs, grad_map, grad_sources [S, 3])."""
    flat = np.asarray(flat, np.float64)
    r = np.asarray(r, np.float64)
    nd = flat.shape[0]
    nb = prob_big.n_det
    rb = np.zeros((nb, nb))
    for f, (r0, c0) in enumerate(dither_windows(dithers, margin)):
        rb[r0:r0 + nd, c0:c0 + nd] += flat * r[f]
    g_c, g_map, g_src = backward(prob_big, coeffs, phase_map, np.asarray(sources, np.float64)[None],
                                 np.ones((nb, nb)), rb[None])
    return g_c, g_map, g_src[0]


def value_and_grad_dithered(prob_big, coeffs, phase_map, sources, flat, data, dithers, margin, kind="poisson",
                            prior_mu=1.0, prior_sigma=0.1):
    """``value_and_grad`` for integer-dithered frames of one scene."""
    B, m = forward_dithered(prob_big, coeffs, phase_map, sources, flat, dithers, margin)
    L, r, gF, bad = loss_grad(m, B, data, flat, kind, prior_mu, prior_sigma)
    g_c, g_map, g_src = backward_dithered(prob_big, coeffs, phase_map, sources, flat, r, dithers, margin)
    return dict(binned=B, model=m, loss=L, r=r, grad_flat=gF, grad_coeffs=g_c, grad_map=g_map,
                grad_sources=g_src, domain=bad)


def intrapixel_grad_dithered(prob_big: OracleProblem, coeffs, phase_map, sources, flat, r, dithers, margin):
    """dL/dK for integer-dithered frames: the enlarged plane's intensity against sum_f (flat r_f) in its window."""
    flat = np.asarray(flat, np.float64)
    r = np.asarray(r, np.float64)
    nd = flat.shape[0]
    nb = prob_big.n_det
    rb = np.zeros((nb, nb))
    for f, (r0, c0) in enumerate(dither_windows(dithers, margin)):
        rb[r0:r0 + nd, c0:c0 + nd] += flat * r[f]
    return intrapixel_grad(prob_big, coeffs, phase_map, np.asarray(sources, np.float64)[None], np.ones((nb, nb)),
                           rb[None])
