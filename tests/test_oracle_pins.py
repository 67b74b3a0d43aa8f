"""Pins of the FP64 oracle to results fixed by mathematics, not by the oracle itself.

Each test ties one part of the oracle to something independent of it: a
brute-force DFT, a library FFT, Parseval's theorem, the Airy closed forms,
the DFT shift theorem, symmetry invariances, the adjoint identity, Euler's
theorem for the flux, library log-likelihoods and central finite
differences. A dropped term, a wrong sign or index, or a transposed operand
anywhere in the oracle fails at least one of them.
"""
import cmath
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle as O
from synth import aperture, zernike_basis, make_workload, keys_bicubic_matrix, noll_to_nm, pixel_centres
from tests.helpers import oracle_problem, rel_l2

RNG = np.random.default_rng(12345)


def _crand(*shape):
    return RNG.normal(size=shape) + 1j * RNG.normal(size=shape)


# --------------------------------------------------------------------------- MFT definition
@pytest.mark.parametrize("ni,no", [(4, 3), (5, 6), (8, 7), (5, 12), (8, 12)])
@pytest.mark.parametrize("centring", ["pixel", "integer"])
def test_mft_matches_brute_force_dft(ni, no, centring):
    lam, dx, du = 550e-9, 0.01, 3.3e-6
    if centring == "pixel":
        x = O.pixel_grid(ni, dx)
        u = O.pixel_grid(no, du)
    else:
        x = (np.arange(ni) - ni // 2) * dx
        u = (np.arange(no) - no // 2) * du
    y, v = x + 0.2 * dx, u - 0.3 * du     # distinct row/column coordinates catch a swapped side
    P = _crand(ni, ni)
    scale = dx * du / lam
    got = O.focal_field(P, x, y, u, v, lam, scale)
    want = np.zeros((no, no), complex)
    for k in range(no):
        for l in range(no):
            acc = 0j
            for m in range(ni):
                for n in range(ni):
                    acc += P[m, n] * cmath.exp(-2j * math.pi * (y[m] * v[k] + x[n] * u[l]) / lam)
            want[k, l] = scale * acc
    assert rel_l2(got, want) < 1e-13


@pytest.mark.parametrize("ni,no", [(16, 32), (16, 20), (24, 48)])
def test_mft_equals_zero_padded_fft_at_nyquist(ni, no):
    lam, dx = 700e-9, 0.5 / ni
    npad = 2 * ni
    du = lam / (npad * dx)
    x = np.arange(ni) * dx                  # phase origin on the first pupil sample
    u = (np.arange(no) - no // 2) * du
    P = _crand(ni, ni)
    got = O.focal_field(P, x, x, u, u, lam, dx * du / lam)
    pad = np.zeros((npad, npad), complex)
    pad[:ni, :ni] = P
    Fs = np.fft.fftshift(np.fft.fft2(pad))
    lo = npad // 2 - no // 2
    want = Fs[lo:lo + no, lo:lo + no] / npad
    assert rel_l2(got, want) < 1e-12


def test_parseval_unit_power_on_full_period_grid():
    w = make_workload("c2", n_pupil=32, n_focal=64, oversample=4, n_wavelengths=1, noll=tuple(range(2, 12)))
    prob = oracle_problem(w)
    lam = prob.wavelengths[0]
    x = O.pixel_grid(32, prob.dx)
    u = O.pixel_grid(64, lam / (64 * prob.dx))
    opd = O.opd_map(prob.zbasis, np.asarray(w.coeffs_true, float))
    P = O.pupil_field(prob.transmission, opd, x, x, 1e-6, -2e-6, lam)
    assert abs(np.sum(np.abs(P) ** 2) - 1.0) < 1e-14
    E = O.focal_field(P, x, x, u, u, lam, prob.dx * (lam / (64 * prob.dx)) / lam)
    assert abs(np.sum(np.abs(E) ** 2) - 1.0) < 1e-13


# --------------------------------------------------------------------------- Airy closed forms
def _radial_profile(ni, eps, no=129, nyq_frac=0.25):
    D, lam = 0.5, 600e-9
    A = aperture(ni, D, obstruction=eps)
    dx = D / ni
    du = nyq_frac * lam / D
    x = O.pixel_grid(ni, dx)
    u = O.pixel_grid(no, du)
    P = O.pupil_field(A, np.zeros_like(A), x, x, 0.0, 0.0, lam)
    E = O.focal_field(P, x, x, u, u, lam, dx * du / lam)
    I = np.abs(E) ** 2
    c = (no - 1) // 2
    v = np.pi * D * u / lam
    return A, dx, du, lam, I, I[c, :], v


def _airy(v, eps):
    v = np.where(v == 0, 1e-300, v)
    a = 2 * special.j1(v) / v
    if eps > 0:
        a = a - eps ** 2 * 2 * special.j1(eps * v) / (eps * v)
    return a ** 2 / (1 - eps ** 2) ** 2


@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_airy_profile_converges_with_pupil_sampling(eps):
    errs = []
    for ni in (64, 128, 256):
        _, _, _, _, _, cut, v = _radial_profile(ni, eps)
        errs.append(np.max(np.abs(cut / cut.max() - _airy(v, eps))))
    # grey-edge discretisation error: small at every sampling, and below the coarsest
    # one's once the pupil is refined (a wrong angular scale or normalisation gives O(1))
    assert max(errs) < 1e-3
    assert errs[1] < errs[0] and errs[2] < errs[0]


def test_airy_first_zero_and_exact_peak():
    A, dx, du, lam, I, cut, v = _radial_profile(256, 0.0, no=257, nyq_frac=1 / 16)
    c = 128
    peak = (dx * du / lam) ** 2 * A.sum() ** 2 / np.sum(A ** 2)
    assert abs(I[c, c] - peak) / peak < 1e-13
    # first dark ring at 1.21967 lambda/D (sampled at lambda/(16 D))
    theta = (np.arange(257) - 128) * du
    k = np.argmin(np.abs(theta - 1.21967 * lam / 0.5))
    assert cut[k] / cut[c] < 2e-3


# --------------------------------------------------------------------------- shift theorem / tilt
def test_source_offset_equals_shifted_grid_and_moves_peak_to_plus_alpha():
    w = make_workload("c2", n_pupil=48, n_focal=64, oversample=4, n_wavelengths=1, noll=tuple(range(2, 12)))
    prob = oracle_problem(w)
    lam = prob.wavelengths[0]
    x = O.pixel_grid(48, prob.dx)
    u = O.pixel_grid(64, prob.focal_pixel)
    opd = O.opd_map(prob.zbasis, np.asarray(w.coeffs_true, float))
    c = prob.dx * prob.focal_pixel / lam
    alpha, beta = 0.37 * prob.focal_pixel * 5, -1.3 * prob.focal_pixel
    Ea = O.focal_field(O.pupil_field(prob.transmission, opd, x, x, alpha, beta, lam), x, x, u, u, lam, c)
    E0 = O.focal_field(O.pupil_field(prob.transmission, opd, x, x, 0.0, 0.0, lam), x, x, u - alpha, u - beta, lam, c)
    assert rel_l2(np.abs(Ea) ** 2, np.abs(E0) ** 2) < 1e-12
    # integer shift by k focal pixels along +x: array translated by +k columns on the overlap
    prob_clear = np.ones_like(prob.transmission)
    k = 3
    P0 = O.pupil_field(prob_clear * prob.transmission, np.zeros_like(opd), x, x, 0.0, 0.0, lam)
    Pk = O.pupil_field(prob_clear * prob.transmission, np.zeros_like(opd), x, x, k * prob.focal_pixel, 0.0, lam)
    I0 = np.abs(O.focal_field(P0, x, x, u, u, lam, c)) ** 2
    Ik = np.abs(O.focal_field(Pk, x, x, u, u, lam, c)) ** 2
    assert rel_l2(Ik[:, k:], I0[:, :-k]) < 1e-12
    assert np.unravel_index(np.argmax(Ik), Ik.shape)[1] - np.unravel_index(np.argmax(I0), I0.shape)[1] == k


@pytest.mark.parametrize("noll,axis", [(2, 0), (3, 1)])
def test_tilt_zernike_equals_source_offset(noll, axis):
    # binary aperture (no grey edge outside the unit disk) so that Z2 = 2x/R on every lit pixel
    D, ni, lam = 0.5, 64, 600e-9
    A = aperture(ni, D, supersample=1)
    Z = zernike_basis([noll], ni, D)
    x = O.pixel_grid(ni, D / ni)
    du = lam / (2 * D) / 2
    u = O.pixel_grid(64, du)
    coef = 37e-9
    shift = 4.0 * coef / D          # Noll Z2 = 2 rho cos(theta) = 2x/R, R = D/2
    P_z = O.pupil_field(A, O.opd_map(Z, [coef]), x, x, 0.0, 0.0, lam)
    ab = (shift, 0.0) if axis == 0 else (0.0, shift)
    P_s = O.pupil_field(A, np.zeros_like(A), x, x, ab[0], ab[1], lam)
    c = (D / ni) * du / lam
    Iz = np.abs(O.focal_field(P_z, x, x, u, u, lam, c)) ** 2
    Is = np.abs(O.focal_field(P_s, x, x, u, u, lam, c)) ** 2
    assert rel_l2(Iz, Is) < 1e-12


# --------------------------------------------------------------------------- invariances
def test_piston_leaves_psf_and_has_zero_gradient():
    D, ni = 0.5, 48
    w = make_workload("c1", n_pupil=ni, n_focal=48, oversample=2)
    A = aperture(ni, D, supersample=1)
    Z = zernike_basis([1, 4, 7, 8], ni, D)
    prob = O.OracleProblem.from_arrays(ni, 48, 2, D, w.problem.focal_pixel, w.problem.wavelengths,
                                       w.problem.weights, A, Z)
    coeffs = np.array([0.0, 30e-9, -20e-9, 15e-9])
    src = np.array([[[1e-7, -2e-7, 1e6]]])
    flat = np.ones((24, 24))
    B0, m0 = O.forward(prob, coeffs, None, src, flat)
    B1, m1 = O.forward(prob, coeffs + np.array([55e-9, 0, 0, 0]), None, src, flat)
    assert rel_l2(B1, B0) < 1e-12
    data = np.random.default_rng(1).poisson(m0 * 1.1).astype(float)
    out = O.value_and_grad(prob, coeffs, None, src, flat, data)
    g = out["grad_coeffs"]
    assert abs(g[0]) < 1e-12 * np.linalg.norm(g[1:])


def test_even_modes_have_sign_ambiguity_odd_modes_do_not():
    D, ni, lam = 0.5, 64, 600e-9
    A = aperture(ni, D, obstruction=0.3, spider_px=2.0)
    np.testing.assert_array_equal(A, A[::-1, ::-1])
    x = O.pixel_grid(ni, D / ni)
    du = lam / (2 * D) / 3
    u = O.pixel_grid(60, du)
    c = (D / ni) * du / lam
    even = [4, 5, 6, 11, 12, 13]
    assert all(noll_to_nm(j)[1] % 2 == 0 for j in even)
    Ze = zernike_basis(even, ni, D)
    ce = np.array([40, -25, 30, 20, -15, 10]) * 1e-9
    I = lambda Z, cc: np.abs(O.focal_field(O.pupil_field(A, O.opd_map(Z, cc), x, x, 0, 0, lam), x, x, u, u, lam, c)) ** 2
    assert rel_l2(I(Ze, ce), I(Ze, -ce)) < 1e-12
    Zo = zernike_basis([7, 8], ni, D)
    co = np.array([40e-9, -25e-9])
    assert rel_l2(I(Zo, co), I(Zo, -co)) > 1e-3


def test_adjoint_dot_product():
    x = O.pixel_grid(12, 0.04)
    y = x * 1.01
    u = O.pixel_grid(17, 2e-6)
    v = u + 1e-7
    lam, sc = 600e-9, 0.04 * 2e-6 / 600e-9
    X = _crand(12, 12)
    Yc = _crand(17, 17)
    lhs = np.vdot(O.focal_field(X, x, y, u, v, lam, sc), Yc)
    rhs = np.vdot(X, O.focal_field_adjoint(Yc, x, y, u, v, lam, sc))
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_binning_matrix_form_and_adjoint():
    Q, nd = 3, 7
    I = RNG.random((Q * nd, Q * nd))
    R = np.kron(np.eye(nd), np.ones((1, Q)))
    np.testing.assert_allclose(O.bin_detector(I, Q), R @ I @ R.T, rtol=1e-14)
    kx = 1.0 + 0.005 * (np.arange(Q) - 1.0) / 2.0
    K = np.tile(kx, (Q, 1))
    Rk = R * np.tile(kx, nd)[None, :]
    np.testing.assert_allclose(O.bin_detector(I, Q, K), R @ I @ Rk.T, rtol=1e-14)
    g = RNG.random((nd, nd))
    assert abs(np.vdot(O.bin_detector(I, Q, K), g) - np.vdot(I, O.expand_detector(g, Q, K))) < 1e-12


# --------------------------------------------------------------------------- loss
def test_poisson_and_prior_match_library_log_densities():
    m = RNG.uniform(0.5, 400.0, size=(2, 5, 5))
    d = RNG.poisson(m).astype(float)
    B = m / 1.07
    Fl = np.full((5, 5), 1.07) + RNG.normal(0, 0.02, (5, 5))
    m = Fl[None] * B
    mu, sig = 1.0, 0.05
    L, r, gF, bad = O.loss_grad(m, B, d, Fl, "poisson", mu, sig)
    want = (-np.sum(stats.poisson.logpmf(d, m)) - np.sum(special.gammaln(d + 1))
            - np.sum(stats.norm.logpdf(Fl, mu, sig)) - Fl.size * math.log(sig * math.sqrt(2 * math.pi)))
    assert abs(L - want) / abs(want) < 1e-12
    assert not bad
    Lc, rc, _, _ = O.loss_grad(m, B, d, Fl, "chi2", mu, sig)
    wgt = np.maximum(d, 1.0)
    want_c = (-np.sum(stats.norm.logpdf(m, d, np.sqrt(wgt))) - np.sum(0.5 * np.log(2 * math.pi * wgt))
              - np.sum(stats.norm.logpdf(Fl, mu, sig)) - Fl.size * math.log(sig * math.sqrt(2 * math.pi)))
    assert abs(Lc - want_c) / abs(want_c) < 1e-12


def test_loss_value_brute_force_fsum():
    w = make_workload("c1")
    prob = oracle_problem(w)
    B, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
    w = w.with_data(m)
    B, m = O.forward(prob, w.coeffs, None, w.sources, w.flat)
    L, r, gF, _ = O.loss_grad(m, B, w.data, w.flat, "poisson", 1.0, 0.05)
    terms = [float(mm) - float(dd) * math.log(float(mm)) for mm, dd in zip(m.ravel(), w.data.ravel())]
    terms += [(float(f) - 1.0) ** 2 / (2 * 0.05 ** 2) for f in w.flat.ravel()]
    assert abs(L - math.fsum(terms)) <= 1e-14 * abs(L) + 1e-14 * math.fsum(abs(t) for t in terms)


# --------------------------------------------------------------------------- gradients
def _fd(f, x0, h):
    """4-point central difference (Richardson): error O(h^4)."""
    return (-f(x0 + 2 * h) + 8 * f(x0 + h) - 8 * f(x0 - h) + f(x0 - 2 * h)) / (12 * h)


def _setup_small(name, **ov):
    w = make_workload(name, **ov)
    prob = oracle_problem(w)
    B, m = O.forward(prob, w.coeffs_true, w.map_true, w.sources_true, w.flat_true)
    w = w.with_data(m)
    return w, prob


SMALL = {
    "c1": dict(n_pupil=32, n_focal=32),
    "c3": dict(n_pupil=24, n_focal=27, n_wavelengths=2, n_frames=2, noll=tuple(range(2, 8))),
    "c5": dict(n_pupil=24, n_focal=28, n_wavelengths=2, n_frames=2, noll=tuple(range(2, 6)), n_map=6),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("kind", ["poisson", "chi2"])
def test_all_gradients_match_central_differences(name, kind):
    w, prob = _setup_small(name, **SMALL[name])
    mu, sig = w.prior_mu, w.prior_sigma
    # a point away from both the truth and the unaberrated start
    rng = np.random.default_rng(7)
    coeffs = np.asarray(w.coeffs_true, float) * 0.6
    pmap = None if w.map_true is None else np.asarray(w.map_true, float) * 0.5
    src = np.asarray(w.sources, float)
    flat = np.asarray(w.flat_true, float) + rng.normal(0, 0.01, w.flat_true.shape)
    data = w.data

    def L(c=coeffs, pm=pmap, s=src, fl=flat):
        B, m = O.forward(prob, c, pm, s, fl)
        return O.loss_grad(m, B, data, fl, kind, mu, sig)[0]

    out = O.value_and_grad(prob, coeffs, pmap, src, flat, data, kind, mu, sig)
    # Zernike block (h = 1e-3 nm)
    fd = np.array([_fd(lambda t: L(c=coeffs + t * np.eye(len(coeffs))[j]), 0.0, 1e-12) for j in range(len(coeffs))])
    assert rel_l2(out["grad_coeffs"], fd) < 1e-6
    # positions (h = 1e-4 focal px) and fluxes (h = 1e-6 phi)
    pix = prob.focal_pixel
    g = out["grad_sources"]
    fdp = np.zeros_like(g)
    for f in range(src.shape[0]):
        for s in range(src.shape[1]):
            for k, h in ((0, 1e-4 * pix), (1, 1e-4 * pix), (2, 1e-6 * src[f, s, 2])):
                def Ls(t, f=f, s=s, k=k):
                    s2 = src.copy()
                    s2[f, s, k] += t
                    return L(s=s2)
                fdp[f, s, k] = _fd(Ls, 0.0, h)
    assert rel_l2(g[..., :2], fdp[..., :2]) < 1e-6
    assert rel_l2(g[..., 2], fdp[..., 2]) < 1e-6
    # flat field (h = 1e-4) on a few pixels
    idx = rng.choice(flat.size, 8, replace=False)
    fdF = []
    for i in idx:
        e = np.zeros(flat.size)
        e[i] = 1.0
        fdF.append(_fd(lambda t: L(fl=flat + t * e.reshape(flat.shape)), 0.0, 1e-4))
    assert rel_l2(out["grad_flat"].ravel()[idx], np.array(fdF)) < 1e-7
    if pmap is not None:
        fdm = np.zeros_like(pmap)
        for a in range(pmap.shape[0]):
            for b in range(pmap.shape[1]):
                e = np.zeros_like(pmap)
                e[a, b] = 1.0
                fdm[a, b] = _fd(lambda t: L(pm=pmap + t * e), 0.0, 1e-12)
        assert rel_l2(out["grad_map"], fdm) < 1e-6


def test_flux_gradient_euler_identity():
    w, prob = _setup_small("c3", **SMALL["c3"])
    src = np.asarray(w.sources, float)
    flat = np.asarray(w.flat_true, float)
    out = O.value_and_grad(prob, w.coeffs, None, src, flat, w.data, "poisson", w.prior_mu, w.prior_sigma)
    r = out["r"]
    for s in range(src.shape[1]):
        only = src.copy()
        keep = np.zeros(src.shape[1])
        keep[s] = 1.0
        only[..., 2] *= keep[None, :]
        _, m_s = O.forward(prob, w.coeffs, None, only, flat)
        for f in range(src.shape[0]):
            lhs = src[f, s, 2] * out["grad_sources"][f, s, 2]
            rhs = np.sum(r[f] * m_s[f])
            assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(r[f] * m_s[f]))


def test_sampled_binned_pixels_match_full_forward():
    w, prob = _setup_small("c3", **SMALL["c3"])
    B, _ = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
    px = [(0, 0), (4, 5), (8, 8), (2, 7)]
    got = O.binned_pixels(prob, w.coeffs_true, None, w.sources_true, 1, px)
    want = np.array([B[1, p, q] for p, q in px])
    np.testing.assert_allclose(got, want, rtol=1e-13)


# --------------------------------------------------------------------------- input generators
def test_noll_table_and_zernike_orthonormality():
    table = {1: (0, 0), 2: (1, 1), 3: (1, -1), 4: (2, 0), 5: (2, -2), 6: (2, 2), 7: (3, -1), 8: (3, 1),
             9: (3, -3), 10: (3, 3), 11: (4, 0), 12: (4, 2), 13: (4, -2), 14: (4, 4), 15: (4, -4), 22: (6, 0)}
    for j, nm in table.items():
        assert noll_to_nm(j) == nm
    Z = zernike_basis(list(range(1, 22)), 256, 2.0)
    inside = np.hypot(*np.meshgrid(pixel_centres(256, 2 / 256), pixel_centres(256, 2 / 256))) <= 1.0
    G = np.einsum("imn,jmn->ij", Z[:, inside][:, None, :], Z[:, inside][:, None, :]) / inside.sum()
    assert np.max(np.abs(G - np.eye(21))) < 2e-2
    # Z2 is exactly 2x/R on the disk
    x = pixel_centres(256, 2 / 256)
    X, _ = np.meshgrid(x, x)
    np.testing.assert_allclose(Z[1][inside], (2 * X)[inside], rtol=0, atol=1e-13)


def test_bicubic_matrix_reproduces_quadratics_in_interior():
    B = keys_bicubic_matrix(96, 10, 0.5)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    xn = pixel_centres(10, 0.05)
    xp = pixel_centres(96, 0.5 / 96)
    q = lambda t: 3.0 + 2.0 * t - 7.0 * t ** 2
    interior = (xp > xn[1]) & (xp < xn[-2])
    np.testing.assert_allclose((B @ q(xn))[interior], q(xp)[interior], atol=1e-12)


def _dither_case():
    ni, nd, Q, margin = 16, 6, 2, 2
    D = 0.5
    pix = 600e-9 / (2 * D)
    lam = np.array([550e-9, 650e-9])
    wts = np.array([0.5, 0.5])
    trans = aperture(ni, D, 0.3, 1.0)
    Z = zernike_basis([4, 5, 6, 7, 8], ni, D)
    rng = np.random.default_rng(41)
    K = 1.0 + 0.05 * rng.normal(size=(Q, Q))
    small = O.OracleProblem.from_arrays(ni, Q * nd, Q, D, pix / Q, lam, wts, trans, Z, None, K)
    big = O.OracleProblem.from_arrays(ni, Q * (nd + 2 * margin), Q, D, pix / Q, lam, wts, trans, Z, None, K)
    pos = np.array([[0.4, -0.7, 3e4], [-1.1, 0.6, 1e4]])
    pos[:, :2] *= pix
    dithers = np.array([[0, 0], [2, -1], [-2, 2], [1, 0]])
    coeffs = 30e-9 * rng.normal(size=5)
    flat = 1.0 + 0.05 * rng.normal(size=(nd, nd))
    per_frame = np.repeat(pos[None], len(dithers), axis=0)
    per_frame[:, :, 0] += dithers[:, 0][:, None] * pix
    per_frame[:, :, 1] += dithers[:, 1][:, None] * pix
    return small, big, pos, per_frame, dithers, margin, coeffs, flat, rng


def test_dithered_frames_from_enlarged_plane_equal_per_frame_model():
    # Section 3's integer dithers: a window of one enlarged plane equals the frame
    # computed with the dither added to every star's position (shift theorem on the grid).
    small, big, pos, per_frame, dithers, margin, coeffs, flat, _ = _dither_case()
    Bd, md = O.forward_dithered(big, coeffs, None, pos, flat, dithers, margin)
    Bs, ms = O.forward(small, coeffs, None, per_frame, flat)
    assert rel_l2(Bd, Bs) < 1e-12
    assert rel_l2(md, ms) < 1e-12


def test_dithered_gradients_equal_frame_sums_of_per_frame_gradients():
    small, big, pos, per_frame, dithers, margin, coeffs, flat, rng = _dither_case()
    _, m = O.forward(small, coeffs, None, per_frame, flat)
    data = rng.poisson(m).astype(np.float64)
    a = O.value_and_grad_dithered(big, coeffs, None, pos, flat, data, dithers, margin, "poisson", 1.0, 0.05)
    b = O.value_and_grad(small, coeffs, None, per_frame, flat, data, "poisson", 1.0, 0.05)
    assert abs(a["loss"] - b["loss"]) < 1e-12 * abs(b["loss"])
    assert rel_l2(a["r"], b["r"]) < 1e-12
    assert rel_l2(a["grad_flat"], b["grad_flat"]) < 1e-12
    assert rel_l2(a["grad_coeffs"], b["grad_coeffs"]) < 1e-11
    assert rel_l2(a["grad_sources"], b["grad_sources"].sum(axis=0)) < 1e-11


def test_dither_windows_reject_dithers_beyond_the_margin():
    with pytest.raises(ValueError):
        O.dither_windows([[3, 0]], 2)
    assert O.dither_windows([[1, -2]], 2).tolist() == [[4, 1]]


@pytest.mark.parametrize("kind", ["poisson", "chi2"])
def test_intrapixel_gradient_matches_central_differences_and_euler(kind):
    # the binned image is linear in K: central differences of L in each K entry, and
    # sum_ab K dL/dK = sum_f sum_p F r B (Euler)
    w, prob = _setup_small("c3", **SMALL["c3"])
    p = w.eval_params()
    K0 = np.array(prob.intrapixel)
    base = O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, kind, w.prior_mu, w.prior_sigma)
    gK = O.intrapixel_grad(prob, p["coeffs"], None, p["sources"], p["flat"], base["r"])

    def loss_at(K):
        pr = O.OracleProblem(**{**prob.__dict__, "intrapixel": K})
        B, m = O.forward(pr, p["coeffs"], None, p["sources"], p["flat"])
        return O.loss_grad(m, B, w.data, p["flat"], kind, w.prior_mu, w.prior_sigma)[0]

    Q = prob.oversample
    for a, b in [(0, 0), (1, 2), (Q - 1, 0)]:
        def fk(t, a=a, b=b):
            K = K0.copy()
            K[a, b] = t
            return loss_at(K)
        fd = _fd(fk, K0[a, b], 1e-4)
        assert abs(fd - gK[a, b]) <= 1e-6 * max(abs(gK[a, b]), 1e-3 * np.abs(gK).max())
    euler = np.sum(np.asarray(p["flat"], np.float64)[None] * base["r"] * base["binned"])
    assert abs(np.sum(K0 * gK) - euler) <= 1e-10 * np.sum(np.abs(K0 * gK))


def test_dithered_intrapixel_gradient_equals_per_frame_sum():
    small, big, pos, per_frame, dithers, margin, coeffs, flat, rng = _dither_case()
    _, m = O.forward(small, coeffs, None, per_frame, flat)
    data = rng.poisson(m).astype(np.float64)
    ref = O.value_and_grad(small, coeffs, None, per_frame, flat, data, "poisson", 1.0, 0.05)
    a = O.intrapixel_grad_dithered(big, coeffs, None, pos, flat, ref["r"], dithers, margin)
    b = O.intrapixel_grad(small, coeffs, None, per_frame, flat, ref["r"])
    assert rel_l2(a, b) < 1e-11


# --------------------------------------------------------------------------- static phase screen, Fresnel defocus
def _screen_case():
    D, ni, no, lam = 0.5, 24, 30, 600e-9
    A = aperture(ni, D, 0.2, 0.0)
    Z = zernike_basis([4, 7, 8], ni, D)
    opd = O.opd_map(Z, [20e-9, -15e-9, 10e-9])
    x = O.pixel_grid(ni, D / ni)
    du = lam / (2 * D) / 2
    u = O.pixel_grid(no, du)
    return D, ni, lam, A, Z, opd, x, u, (D / ni) * du / lam


def test_constant_phase_screen_is_a_global_phase():
    D, ni, lam, A, Z, opd, x, u, c = _screen_case()
    E0 = O.focal_field(O.pupil_field(A, opd, x, x, 1e-7, -2e-7, lam), x, x, u, u, lam, c)
    Es = O.focal_field(O.pupil_field(A, opd, x, x, 1e-7, -2e-7, lam, np.full((ni, ni), 1.3)), x, x, u, u, lam, c)
    assert rel_l2(Es, E0 * np.exp(1.3j)) < 1e-13


def test_phase_screen_in_radians_equals_the_same_opd_at_one_wavelength():
    # a screen phi acts like an OPD phi * lambda / (2 pi) at that wavelength: pins the unit and the sign
    D, ni, lam, A, Z, opd, x, u, c = _screen_case()
    extra = O.opd_map(Z, [-31e-9, 12e-9, 25e-9])
    Eo = O.focal_field(O.pupil_field(A, opd + extra, x, x, 0.0, 0.0, lam), x, x, u, u, lam, c)
    Es = O.focal_field(O.pupil_field(A, opd, x, x, 0.0, 0.0, lam, 2 * np.pi * extra / lam), x, x, u, u, lam, c)
    assert rel_l2(Es, Eo) < 1e-13


def test_binary_half_wave_screen_flips_the_sign_of_its_region():
    # exp(i pi) = -1 on the plate's region R: by linearity of the transform E = E(P) - 2 E(P restricted to R)
    D, ni, lam, A, Z, opd, x, u, c = _screen_case()
    from synth import binary_phase_screen
    R = binary_phase_screen(ni, np.random.default_rng(7)) > 1.0
    assert 0.2 < R.mean() < 0.8
    scr = np.where(R, np.pi, 0.0)     # exact pi in FP64 (the stand-in itself is FP32)
    P = O.pupil_field(A, opd, x, x, 0.0, 0.0, lam)
    Es = O.focal_field(O.pupil_field(A, opd, x, x, 0.0, 0.0, lam, scr), x, x, u, u, lam, c)
    want = O.focal_field(P, x, x, u, u, lam, c) - 2.0 * O.focal_field(P * R, x, x, u, u, lam, c)
    assert rel_l2(Es, want) < 1e-13


def test_screened_model_gradients_match_central_differences():
    w = make_workload("c1", n_pupil=24, n_focal=16, noll=(2, 4, 7, 8))
    prob = oracle_problem(w)
    from synth import binary_phase_screen
    import dataclasses
    prob = dataclasses.replace(prob, phase_screen=binary_phase_screen(24, np.random.default_rng(3)).astype(np.float64))
    p = w.eval_params()
    _, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
    d = np.round(m)
    ref = O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], d, "poisson", w.prior_mu, w.prior_sigma)
    L = lambda cc, ss: O.value_and_grad(prob, cc, None, ss, p["flat"], d, "poisson", w.prior_mu,
                                        w.prior_sigma)["loss"]
    c0 = np.asarray(p["coeffs"], np.float64)
    s0 = np.asarray(p["sources"], np.float64)
    h = 1e-12
    for j in range(c0.size):
        e = np.zeros_like(c0)
        e[j] = h
        fd = (8 * (L(c0 + e, s0) - L(c0 - e, s0)) - (L(c0 + 2 * e, s0) - L(c0 - 2 * e, s0))) / (12 * h)
        assert abs(fd - ref["grad_coeffs"][j]) < 1e-6 * np.max(np.abs(ref["grad_coeffs"])) + 1e-9
    hp = 1e-4 * w.problem.focal_pixel
    for k in range(2):
        e = np.zeros_like(s0)
        e[0, 0, k] = hp
        fd = (8 * (L(c0, s0 + e) - L(c0, s0 - e)) - (L(c0, s0 + 2 * e) - L(c0, s0 - 2 * e))) / (12 * hp)
        assert abs(fd - ref["grad_sources"][0, 0, k]) < 1e-6 * abs(ref["grad_sources"][0, 0, k]) + 1e-3


def test_fresnel_defocus_basis_matches_angular_spectrum_propagation():
    # Odd pupil, full-period focal grid (N_o = N_pad, du = lambda / (N_pad dx)): the focal field is an exact
    # periodic DFT of the pupil, so propagating it a distance delta by its angular spectrum (paraxial
    # transfer function exp(-i pi lambda delta kappa^2) in this sign convention, where a +alpha tilt images
    # at +alpha) is exact, and must equal the focal field of the pupil with the defocus OPD added.
    from synth import fresnel_defocus_basis
    D, ni, lam, f = 0.5, 33, 600e-9, 8.0
    npad = 66
    dx = D / ni
    du = lam / (npad * dx)
    x = O.pixel_grid(ni, dx)
    u = O.pixel_grid(npad, du)       # u = 0 lies between samples (even N): shifted below by half a pixel
    u = (np.arange(npad) - npad // 2) * du
    A = aperture(ni, D, 0.15, 0.0)
    Z = zernike_basis([4, 7, 8, 11], ni, D)
    opd = O.opd_map(Z, [15e-9, -20e-9, 8e-9, 5e-9])
    c = dx * du / lam
    E0 = O.focal_field(O.pupil_field(A, opd, x, x, 0.0, 0.0, lam), x, x, u, u, lam, c)
    dX = f * du
    kap = np.fft.fftfreq(npad, d=dX)
    for delta in (2e-3, -3.5e-3):
        H = np.exp(-1j * np.pi * lam * delta * (kap[None, :] ** 2 + kap[:, None] ** 2))
        Ed = np.fft.fftshift(np.fft.ifft2(np.fft.fft2(np.fft.ifftshift(E0)) * H))
        B = fresnel_defocus_basis(ni, D, f).astype(np.float64)
        Ep = O.focal_field(O.pupil_field(A, opd + delta * B, x, x, 0.0, 0.0, lam), x, x, u, u, lam, c)
        assert np.max(np.abs(delta * B)) > 0.2 * lam          # a visible defocus, not a no-op
        assert rel_l2(Ed, Ep) < 1e-5   # FP32 basis values
        assert rel_l2(np.abs(Ed) ** 2, np.abs(E0) ** 2) > 0.1


# --------------------------------------------------------------------------- one intra-pixel kernel per pixel
def test_kernel_on_focal_grid_layout_brute_force():
    rng = np.random.default_rng(5)
    n, Q = 3, 4
    K = rng.normal(size=(n, n, Q, Q))
    want = np.zeros((n * Q, n * Q))
    for p in range(n):
        for q in range(n):
            for a in range(Q):
                for b in range(Q):
                    want[Q * p + a, Q * q + b] = K[p, q, a, b]
    assert np.array_equal(O.kernel_on_focal_grid(K, n, Q), want)
    Ks = rng.normal(size=(Q, Q))
    assert np.array_equal(O.kernel_on_focal_grid(np.broadcast_to(Ks, (n, n, Q, Q)), n, Q),
                          O.kernel_on_focal_grid(Ks, n, Q))


def _per_pixel_case():
    import dataclasses
    w, prob = _setup_small("c3", **SMALL["c3"])
    n, Q = prob.n_det, prob.oversample
    rng = np.random.default_rng(17)
    Kp = np.asarray(prob.intrapixel)[None, None] * (1 + 0.02 * rng.normal(size=(n, n, Q, Q)))
    return w, prob, dataclasses.replace(prob, intrapixel=Kp), Kp


def test_per_pixel_kernel_equal_everywhere_reduces_to_the_shared_kernel():
    import dataclasses
    w, prob, _, _ = _per_pixel_case()
    n, Q = prob.n_det, prob.oversample
    same = dataclasses.replace(prob, intrapixel=np.broadcast_to(prob.intrapixel, (n, n, Q, Q)).copy())
    p = w.eval_params()
    a = O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson", w.prior_mu,
                         w.prior_sigma)
    b = O.value_and_grad(same, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson", w.prior_mu,
                         w.prior_sigma)
    for k in ("binned", "grad_flat", "grad_coeffs", "grad_sources"):
        assert rel_l2(b[k], a[k]) < 1e-13, k
    gs = O.intrapixel_grad(prob, p["coeffs"], None, p["sources"], p["flat"], a["r"])
    gp = O.intrapixel_grad(same, p["coeffs"], None, p["sources"], p["flat"], a["r"])
    assert gp.shape == (n, n, Q, Q)
    assert rel_l2(gp.sum(axis=(0, 1)), gs) < 1e-13


def test_per_pixel_kernel_gradient_central_differences_and_euler():
    w, _, prob, Kp = _per_pixel_case()
    p = w.eval_params()
    base = O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson", w.prior_mu,
                            w.prior_sigma)
    g = O.intrapixel_grad(prob, p["coeffs"], None, p["sources"], p["flat"], base["r"])

    def loss_at(K):
        pr = O.OracleProblem(**{**prob.__dict__, "intrapixel": K})
        B, m = O.forward(pr, p["coeffs"], None, p["sources"], p["flat"])
        return O.loss_grad(m, B, w.data, p["flat"], "poisson", w.prior_mu, w.prior_sigma)[0]

    n, Q = prob.n_det, prob.oversample
    peak = np.unravel_index(np.argmax(np.abs(g)), g.shape)
    for idx in [peak, (n // 2, n // 3, 0, Q - 1), (1, n - 2, Q - 1, 1)]:
        def fk(t, idx=idx):
            K = Kp.copy()
            K[idx] = t
            return loss_at(K)
        fd = _fd(fk, Kp[idx], 1e-4)
        assert abs(fd - g[idx]) <= 1e-6 * max(abs(g[idx]), 1e-3 * np.abs(g).max()), idx
    euler = np.sum(np.asarray(p["flat"], np.float64)[None] * base["r"] * base["binned"])
    assert abs(np.sum(Kp * g) - euler) <= 1e-10 * np.sum(np.abs(Kp * g))


@pytest.mark.parametrize("ni,no", [(8, 6), (7, 9), (33, 39), (16, 5), (1, 4)])
def test_centred_grid_dft_folds_to_pair_sums_and_differences(ni, no):
    """The identity the GPU path's symmetric fold rests on, on the oracle's own grids (Section 3's
    pixel-centred samples): reversing either index of the DFT matrix conjugates it, so the product
    with any X equals, row a and its mirror, P +- iR with P = Re(M) (X + X_rev) and R = Im(M) (X - X_rev)
    over half the depth; the middle sample of an odd length enters once."""
    rng = np.random.default_rng(ni * 100 + no)
    lam = 6e-7
    x = O.pixel_grid(ni, 0.5 / ni)
    u = O.pixel_grid(no, 1.5e-7)
    M = O.dft_matrix(x, u, lam)
    assert np.max(np.abs(M[:, ::-1] - np.conj(M))) < 1e-13
    assert np.max(np.abs(M[::-1, :] - np.conj(M))) < 1e-13
    X = rng.normal(size=(ni, 3)) + 1j * rng.normal(size=(ni, 3))
    hk, ha = (ni + 1) // 2, (no + 1) // 2
    Xm = X[::-1].copy()
    if ni % 2:
        Xm[hk - 1] = 0.0   # the middle sample is its own mirror
    Xe, Xo = X[:hk] + Xm[:hk], X[:hk] - Xm[:hk]
    P = M[:ha, :hk].real @ Xe
    R = M[:ha, :hk].imag @ Xo
    dense = M @ X
    scale = np.max(np.abs(dense))
    assert np.max(np.abs((P + 1j * R) - dense[:ha])) < 1e-12 * scale
    mirror = no - 1 - np.arange(ha)
    assert np.max(np.abs((P - 1j * R) - dense[mirror])) < 1e-12 * scale
