"""The paper's printed description of its own run (Section 3), against the oracle.

The paper fits 20 stars seen through 3 wavelengths with 7 Zernike terms (Noll
4-10, the first four radial orders without piston, tip and tilt) and one free
response per pixel of a 1024 x 1024 detector, and states the resulting
parameter counts, the PSF count and that its 20-pixel dithers (12 mas pixels)
span about one lambda/D. Here the oracle's value-and-gradient is run on a
problem of that structure at a tiny grid size, and its gradient blocks must
have exactly the printed sizes (the detector block scales as N_det^2).
"""
import os

import numpy as np

import oracle as O
from synth import aperture, noll_to_nm, zernike_basis

HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "paper_run.txt")):
        line = line.split("#")[0].split()
        if line:
            out[line[0]] = [float(v) for v in line[1:]]
    return out


def test_parameter_and_psf_counts_match_the_paper():
    g = golden()
    lam = np.array(g["wavelengths_nm"]) * 1e-9
    assert np.allclose(lam, np.linspace(545e-9, 645e-9, 3))
    S = int(g["stars"][0])
    noll = tuple(int(j) for j in g["zernike_noll"])
    D = g["diameter_m"][0]
    ni, nd = 16, 8
    trans = aperture(ni, D, 0.2, 0.0)
    Z = zernike_basis(noll, ni, D)
    pix = 595e-9 / (2 * D)
    prob = O.OracleProblem.from_arrays(ni, nd, 1, D, pix, lam, np.full(3, 1 / 3), trans, Z, None, None)
    rng = np.random.default_rng(5)
    src = np.zeros((1, S, 3))
    src[0, :, :2] = rng.uniform(-2, 2, (S, 2)) * pix
    src[0, :, 2] = 1e4
    flat = np.ones((nd, nd))
    coeffs = 20e-9 * rng.normal(size=len(noll))
    _, m = O.forward(prob, coeffs, None, src, flat)
    data = rng.poisson(m).astype(np.float64)
    out = O.value_and_grad(prob, coeffs, None, src, flat, data, "poisson", 1.0, 0.1)
    assert out["grad_sources"][..., :2].size == g["param_positions"][0]
    assert out["grad_sources"][..., 2].size == g["param_fluxes"][0]
    assert out["grad_coeffs"].size == g["param_aberrations"][0]
    assert out["grad_flat"].shape == (nd, nd)
    assert int(g["detector_pixels"][0]) ** 2 == g["param_detector"][0]
    assert S * len(lam) == g["psfs"][0]
    assert np.all(np.isfinite(out["grad_sources"])) and np.all(np.isfinite(out["grad_coeffs"]))


def test_named_zernike_terms_are_the_first_radial_orders_without_piston_tip_tilt():
    g = golden()
    noll = [int(j) for j in g["zernike_noll"]]
    orders = {noll_to_nm(j)[0] for j in range(1, noll[-1] + 1)}
    assert orders == set(range(int(g["zernike_radial_orders_named"][0])))
    assert [noll_to_nm(j)[0] for j in (1, 2, 3)] == [0, 1, 1]
    assert set(noll) == set(range(1, noll[-1] + 1)) - {1, 2, 3}


def test_dither_spans_about_one_lambda_over_d():
    g = golden()
    mas = np.pi / 180 / 3600 / 1000
    dither = g["dither_pixels"][0] * g["detector_pixel_mas"][0] * mas
    lam_over_d = np.mean(g["wavelengths_nm"]) * 1e-9 / g["diameter_m"][0]
    assert abs(dither / lam_over_d - g["dither_lambda_over_d"][0]) < 0.03
