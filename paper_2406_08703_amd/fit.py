"""Staged fit and Laplace errors of the paper's experiment (Section 4) on the library's value and gradient.

The paper recovers star positions, fluxes, Zernike coefficients and every
pixel response by Adam on the posterior (Poisson likelihood plus the
pixel-response prior), in two stages: positions, fluxes and aberrations
first with the pixel-response learning rate at zero, then the pixel
response alone with the rest frozen. Errors come from the Laplace
approximation, the inverse Hessian of the likelihood over positions,
fluxes and aberrations with the pixel response held fixed.

Every value and gradient here is one replay of the library's captured
evaluation (dlx_graph_launch); this module only keeps the optimiser state
and the parametrisation. Parameters are updated in natural units so one
Adam learning rate per group is meaningful: positions in detector pixels,
fluxes as log photons, Zernike coefficients in nanometres, the pixel
response as is. The Hessian is the central difference of the analytic
gradient along each of those parameters.

Usage (the paper's run on synthetic data, integer-dither mode):

    python -m paper_2406_08703_amd.fit [--epochs-psf 100] [--epochs-prf 50] [--decay 1.0]
"""
from __future__ import annotations

import json
import time
from dataclasses import dataclass

import torch

from .psf import CapturedEval, PsfPlan

NM = 1e-9


@dataclass
class FitState:
    """Parameters in natural units (device tensors)."""
    pos_px: torch.Tensor      # [S, 2] star positions in detector pixels
    log_flux: torch.Tensor    # [S] natural log of photons per frame
    coeffs_nm: torch.Tensor   # [Nz] Zernike coefficients in nanometres
    flat: torch.Tensor        # [Nd, Nd] pixel response


class _Adam:
    """Adam (Kingma & Ba 2014) on one tensor, default moments."""

    def __init__(self, like: torch.Tensor, lr: float, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = torch.zeros_like(like, dtype=torch.float64)
        self.v = torch.zeros_like(like, dtype=torch.float64)
        self.t = 0

    def step(self, x: torch.Tensor, g: torch.Tensor):
        self.t += 1
        g = g.to(torch.float64)
        self.m.mul_(self.b1).add_(g, alpha=1 - self.b1)
        self.v.mul_(self.b2).addcmul_(g, g, value=1 - self.b2)
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        x.sub_((self.lr * mh / (vh.sqrt() + self.eps)).to(x.dtype))


class Evaluator:
    """Value and gradient of one problem in integer-dither mode (sources [S, 3]) or with one frame."""

    def __init__(self, plan: PsfPlan, data: torch.Tensor, kind="poisson", prior_mu=1.0, prior_sigma=0.1):
        g = plan.geom
        if not g.dithers and g.n_frames != 1:
            raise ValueError("the fit shares star positions across frames: use integer-dither mode or one frame")
        self.plan = plan
        self.pix = g.focal_pixel * g.oversample
        dev = plan.device
        shp = g.sources_shape
        self.sources = torch.zeros(shp, dtype=torch.float32, device=dev)
        self.coeffs = torch.zeros(max(g.n_zernike, 1), dtype=torch.float32, device=dev)[:g.n_zernike]
        self.flat = torch.ones((g.n_det, g.n_det), dtype=torch.float32, device=dev)
        self.data = data
        self.cap = CapturedEval(plan, self.coeffs if g.n_zernike else None, None, self.sources, self.flat, data,
                                kind, prior_mu, prior_sigma)

    def load(self, st: FitState):
        src = self.sources.view(-1, self.sources.shape[-2], 3)[0] if self.sources.dim() == 3 else self.sources
        src[:, 0:2].copy_((st.pos_px.to(torch.float64) * self.pix).to(torch.float32))
        src[:, 2].copy_(st.log_flux.to(torch.float64).exp().to(torch.float32))
        if self.coeffs.numel():
            self.coeffs.copy_((st.coeffs_nm.to(torch.float64) * NM).to(torch.float32))
        self.flat.copy_(st.flat)

    def __call__(self, st: FitState):
        """(loss, d/dpos_px [S,2], d/dlog_flux [S], d/dcoeffs_nm [Nz], d/dflat) at ``st``."""
        self.load(st)
        o = self.cap.replay()
        gs = o.grad_sources.view(-1, 3) if o.grad_sources.dim() == 2 else o.grad_sources[0]
        flux = st.log_flux.to(torch.float64).exp()
        g_pos = gs[:, 0:2] * self.pix
        g_lf = gs[:, 2] * flux
        g_c = o.grad_zernike[:self.coeffs.numel()] * NM
        return o.loss[0], g_pos, g_lf, g_c, o.grad_flat


def fit_staged(ev: Evaluator, st: FitState, epochs_psf=100, epochs_prf=50, lr_pos=0.05, lr_logflux=0.005,
               lr_nm=1.0, lr_flat=0.005, decay=1.0, log_every=0):
    """Section 4's two stages: positions, fluxes and aberrations with the pixel response fixed, then the pixel
    response alone. Updates ``st`` in place and returns the loss after every epoch. ``decay`` < 1 lowers
    every learning rate geometrically over each stage, to ``decay`` times its start at the stage's last
    epoch (1: constant rates)."""
    hist = []
    opt = dict(pos=_Adam(st.pos_px, lr_pos), lf=_Adam(st.log_flux, lr_logflux), c=_Adam(st.coeffs_nm, lr_nm))

    def scale(opts, e, n):
        f = decay ** (e / max(n - 1, 1))
        for o, lr in opts:
            o.lr = lr * f

    for e in range(epochs_psf):
        scale(((opt["pos"], lr_pos), (opt["lf"], lr_logflux), (opt["c"], lr_nm)), e, epochs_psf)
        L, gp, glf, gc, _ = ev(st)
        hist.append(L.clone())   # on the device: no host wait per epoch
        opt["pos"].step(st.pos_px, gp)
        opt["lf"].step(st.log_flux, glf)
        if gc.numel():
            opt["c"].step(st.coeffs_nm, gc)
        if log_every and e % log_every == 0:
            print(f"psf epoch {e}: loss {float(hist[-1]):.6e}", flush=True)
    oflat = _Adam(st.flat, lr_flat)
    for e in range(epochs_prf):
        scale(((oflat, lr_flat),), e, epochs_prf)
        L, _, _, _, gF = ev(st)
        hist.append(L.clone())
        oflat.step(st.flat, gF)
        if log_every and e % log_every == 0:
            print(f"prf epoch {e}: loss {float(hist[-1]):.6e}", flush=True)
    hist.append(ev(st)[0].clone())
    return torch.stack(hist).cpu().tolist()


def laplace_hessian(ev: Evaluator, st: FitState, h_px=0.05, h_logflux=5e-3, h_nm=0.25):
    """Hessian of the loss over (positions [px], log fluxes, Zernike coefficients [nm]) with the pixel
    response fixed, by central differences of the analytic gradient; symmetrised. Order of the
    parameters: x0, y0, x1, y1, ..., log flux 0..S-1, c_0..c_{Nz-1}."""
    S = st.pos_px.shape[0]
    Nz = st.coeffs_nm.numel()
    n = 3 * S + Nz

    def grad_vec():
        _, gp, glf, gc, _ = ev(st)
        return torch.cat([gp.reshape(-1), glf.reshape(-1), gc.reshape(-1)]).to(torch.float64)

    def bump(i, d):
        if i < 2 * S:
            st.pos_px.view(-1)[i] += d
        elif i < 3 * S:
            st.log_flux[i - 2 * S] += d
        else:
            st.coeffs_nm[i - 3 * S] += d

    H = torch.zeros((n, n), dtype=torch.float64, device=st.pos_px.device)
    for i in range(n):
        h = h_px if i < 2 * S else (h_logflux if i < 3 * S else h_nm)
        bump(i, h)
        gp = grad_vec()
        bump(i, -2 * h)
        gm = grad_vec()
        bump(i, h)
        H[:, i] = (gp - gm) / (2 * h)
    return 0.5 * (H + H.T)


def laplace_errors(H: torch.Tensor) -> torch.Tensor:
    """1-sigma errors from the inverse Hessian (marginalised over every parameter of H)."""
    return torch.linalg.inv(H).diagonal().clamp_min(0).sqrt()


def _main():
    import argparse

    import numpy as np

    from synth import make_dithered_workload
    from .psf import Geometry

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--epochs-psf", type=int, default=100)
    ap.add_argument("--epochs-prf", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--decay", type=float, default=1.0, help="learning-rate factor reached at each stage's end")
    args = ap.parse_args()
    w = make_dithered_workload()
    P = w.problem
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    geom = Geometry(P.n_pupil, P.oversample * w.n_det, P.oversample, tuple(P.wavelengths), tuple(P.weights),
                    P.n_sources, w.n_frames, P.n_zernike, 0, P.diameter, P.focal_pixel,
                    tuple(map(tuple, w.dithers.tolist())), w.margin)
    plan = PsfPlan(geom, dev(w.transmission), dev(w.zbasis), precision=args.precision)
    if w.phase_screen is not None:
        plan.set_phase_screen(dev(w.phase_screen))
    # data: photon noise on the model at the truth, as in the paper's simulation
    _, m_true = plan.forward(dev(w.coeffs_true), None, dev(w.sources_true), dev(w.flat_true))
    gen = torch.Generator(device="cuda").manual_seed(2406)
    data = torch.poisson(m_true.clamp_min(0).double(), generator=gen).float()
    ev = Evaluator(plan, data, "poisson", w.prior_mu, w.prior_sigma)
    pix = P.focal_pixel * P.oversample
    ep = w.eval_params()
    st = FitState(pos_px=dev(ep["sources"][:, :2] / pix).double(), log_flux=dev(np.log(ep["sources"][:, 2])).double(),
                  coeffs_nm=dev(ep["coeffs"] / NM).double(), flat=dev(ep["flat"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = fit_staged(ev, st, args.epochs_psf, args.epochs_prf, decay=args.decay)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    t0 = time.perf_counter()
    H = laplace_hessian(ev, st)
    err = laplace_errors(H).cpu().numpy()
    t_h = time.perf_counter() - t0
    assert plan.sync() == 0
    S = P.n_sources
    truth_px = w.sources_true[:, :2] / pix
    dpos = st.pos_px.cpu().numpy() - truth_px
    print(json.dumps({
        "workload": "the paper's run (integer-dither mode); data: Poisson draw of the model at the truth",
        "precision": args.precision, "epochs": [args.epochs_psf, args.epochs_prf], "lr_decay": args.decay,
        "loss_first": hist[0], "loss_last": hist[-1], "fit_seconds": round(t_fit, 3),
        "ms_per_epoch": round(1e3 * t_fit / (args.epochs_psf + args.epochs_prf), 3),
        "hessian_params": int(H.shape[0]), "hessian_seconds": round(t_h, 3),
        "position_error_px_rms": float(np.sqrt(np.mean(dpos ** 2))),
        "median_position_sigma_px": float(np.median(err[:2 * S])),
        "flux_rel_error_rms": float(np.sqrt(np.mean((np.exp(st.log_flux.cpu().numpy()) / w.sources_true[:, 2] - 1) ** 2))),
        "zernike_error_nm_rms": float(np.sqrt(np.mean((st.coeffs_nm.cpu().numpy() - w.coeffs_true / NM) ** 2))),
        "flat_error_rms": float(np.sqrt(np.mean((st.flat.cpu().numpy() - w.flat_true) ** 2))),
        # residuals in units of their Laplace errors (about 1 at the posterior optimum)
        "position_pull_rms": float(np.sqrt(np.mean((dpos.ravel() / err[:2 * S]) ** 2))),
        "log_flux_pull_rms": float(np.sqrt(np.mean(((st.log_flux.cpu().numpy() - np.log(w.sources_true[:, 2]))
                                                    / err[2 * S:3 * S]) ** 2))),
        "zernike_pull_rms": float(np.sqrt(np.mean(((st.coeffs_nm.cpu().numpy() - w.coeffs_true / NM)
                                                   / err[3 * S:]) ** 2))),
        "initial_position_error_px_rms": float(np.sqrt(np.mean((ep["sources"][:, :2] / pix - truth_px) ** 2))),
    }), flush=True)
    plan.close()


if __name__ == "__main__":
    _main()
