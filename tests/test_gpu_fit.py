"""The staged fit and Laplace errors of Section 4 on the GPU path.

The Hessian over positions, fluxes and aberrations (central differences of
the library's analytic gradient) is compared with the same central
differences of the FP64 oracle's gradient; the staged Adam fit must lower
the loss and pull the star positions to the truth.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from tests.test_gpu_dither import case, oracle_big, plan_for

pytestmark = pytest.mark.gpu

NM = 1e-9
# difference steps: well above the FP32 noise of the gradient, well below the PSF's scale (~20 px)
H_PX, H_LF, H_NM = 0.05, 5e-3, 0.25


def _state(w, params):
    import torch
    from paper_2406_08703_amd.fit import FitState
    pix = w.problem.focal_pixel * w.problem.oversample
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()
    src = np.asarray(params["sources"], np.float64)
    return FitState(pos_px=t(src[:, :2] / pix), log_flux=t(np.log(src[:, 2])),
                    coeffs_nm=t(np.asarray(params["coeffs"], np.float64) / NM),
                    flat=t(params["flat"]).float())


def _oracle_grad(w, big, theta, S, Nz, flat):
    pix = w.problem.focal_pixel * w.problem.oversample
    src = np.zeros((S, 3))
    src[:, :2] = theta[:2 * S].reshape(S, 2) * pix
    src[:, 2] = np.exp(theta[2 * S:3 * S])
    c = theta[3 * S:] * NM
    out = O.value_and_grad_dithered(big, c, None, src, flat, w.data, w.dithers, w.margin, "poisson",
                                    w.prior_mu, w.prior_sigma)
    g = out["grad_sources"]
    return np.concatenate([(g[:, :2] * pix).ravel(), g[:, 2] * src[:, 2], out["grad_coeffs"] * NM])


def test_laplace_hessian_matches_oracle_central_differences():
    """At the truth with noise-free data the Hessian is the Fisher matrix, so it is positive definite and
    the Laplace errors exist (with Poisson data it need not be, away from the fitted optimum)."""
    import torch
    from paper_2406_08703_amd.fit import Evaluator, laplace_errors, laplace_hessian
    from tests.gpu_helpers import dev
    print("laplace hessian", flush=True)
    w, _ = case("q1")
    _, m = O.forward_dithered(oracle_big(w), w.coeffs_true, None, w.sources_true, w.flat_true, w.dithers,
                              w.margin)
    w = dataclasses.replace(w, data=np.asarray(m, np.float32))
    S, Nz = w.problem.n_sources, w.problem.n_zernike
    plan = plan_for(w)
    ev = Evaluator(plan, dev(w.data), "poisson", w.prior_mu, w.prior_sigma)
    st = _state(w, w.truth_params())
    H = laplace_hessian(ev, st, h_px=H_PX, h_logflux=H_LF, h_nm=H_NM).cpu().numpy()
    err = laplace_errors(torch.from_numpy(H)).numpy()
    assert plan.sync() == 0
    plan.close()
    big = oracle_big(w)
    theta = np.concatenate([st.pos_px.cpu().numpy().ravel(), st.log_flux.cpu().numpy(), st.coeffs_nm.cpu().numpy()])
    n = theta.size
    Href = np.zeros((n, n))
    flat = st.flat.cpu().numpy().astype(np.float64)
    for i in range(n):
        h = H_PX if i < 2 * S else (H_LF if i < 3 * S else H_NM)
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        Href[:, i] = (_oracle_grad(w, big, tp, S, Nz, flat) - _oracle_grad(w, big, tm, S, Nz, flat)) / (2 * h)
    Href = 0.5 * (Href + Href.T)
    rel = np.linalg.norm(H - Href) / np.linalg.norm(Href)
    err_ref = np.sqrt(np.diag(np.linalg.inv(Href)))
    erel = np.max(np.abs(err / err_ref - 1))
    print(f"hessian rel={rel:.2e}, laplace error max rel={erel:.2e}", flush=True)
    assert rel < 1e-3
    assert np.all(np.linalg.eigvalsh(Href) > 0)
    assert np.all(np.isfinite(err)) and erel < 1e-2


def _resolved_case():
    """Four stars on a 64-pixel detector of 60 mas pixels (lambda/D about 4 pixels), at least 8 pixels
    apart, Poisson data at the truth; unlike the small parity case, whose PSF is wider than the star
    field, the positions here are constrained to a few thousandths of a pixel."""
    from synth import make_dithered_workload
    w = make_dithered_workload(n_pupil=48, n_det=64, margin=6, n_sources=4, det_pixel_mas=60.0,
                               dithers=((0, 0), (6, 6), (6, -6), (-6, 6), (-6, -6)), mask=False)
    _, m = O.forward_dithered(oracle_big(w), w.coeffs_true, None, w.sources_true, w.flat_true, w.dithers,
                              w.margin)
    return w.with_data(m)


def test_staged_fit_recovers_positions_and_lowers_the_loss():
    from paper_2406_08703_amd.fit import Evaluator, fit_staged
    from tests.gpu_helpers import dev
    print("staged fit", flush=True)
    w = _resolved_case()
    pix = w.problem.focal_pixel * w.problem.oversample
    plan = plan_for(w)
    ev = Evaluator(plan, dev(w.data), "poisson", w.prior_mu, w.prior_sigma)
    st = _state(w, w.eval_params())
    truth = w.sources_true[:, :2] / pix
    e0 = np.sqrt(np.mean((st.pos_px.cpu().numpy() - truth) ** 2))
    hist = fit_staged(ev, st, epochs_psf=80, epochs_prf=20)
    assert plan.sync() == 0
    plan.close()
    e1 = np.sqrt(np.mean((st.pos_px.cpu().numpy() - truth) ** 2))
    print(f"position rms {e0:.3f} -> {e1:.3f} px, loss {hist[0]:.6e} -> {hist[-1]:.6e}", flush=True)
    assert hist[-1] < hist[0]
    assert e1 < 0.1 * e0
