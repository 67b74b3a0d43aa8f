"""Run the HIP path through the C ABI on a synthetic workload (GPU tests only)."""
import numpy as np
import torch

from paper_2406_08703_amd import Geometry, PsfPlan


def geometry(w) -> Geometry:
    P = w.problem
    return Geometry(P.n_pupil, P.n_focal, P.oversample, tuple(P.wavelengths), tuple(P.weights), P.n_sources,
                    P.n_frames, P.n_zernike, P.n_map, P.diameter, P.focal_pixel)


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def make_plan(w, precision="fp32", workspace_limit=0, autotune=True, seed_pass=False, dense_mft=False):
    return PsfPlan(geometry(w), dev(w.transmission), dev(w.zbasis) if w.problem.n_zernike else None,
                   dev(w.map_basis), dev(w.intrapixel), precision=precision, workspace_limit=workspace_limit,
                   autotune=autotune, seed_pass=seed_pass, dense_mft=dense_mft)


def run_gpu(w, params=None, kind="poisson", plan=None, precision="fp32"):
    """Forward, loss and backward on the GPU; returns FP64 numpy arrays."""
    params = params or w.eval_params()
    own = plan is None
    plan = plan or make_plan(w, precision)
    c = dev(params["coeffs"])
    pm = dev(params["phase_map"])
    s = dev(params["sources"])
    fl = dev(params["flat"])
    d = dev(w.data)
    B, m = plan.forward(c, pm, s, fl)
    L, r, gF = plan.loss_grad(m, B, d, fl, kind, w.prior_mu, w.prior_sigma)
    gz, gm, gs = plan.backward(c, pm, s, fl, r)
    status = plan.sync()
    out = dict(binned=B, model=m, loss=L[0], r=r, grad_flat=gF, grad_coeffs=gz, grad_map=gm, grad_sources=gs)
    out = {k: (None if v is None else v.detach().cpu().numpy().astype(np.float64)) for k, v in out.items()}
    out["loss"] = float(out["loss"])
    out["status"] = status
    if own:
        plan.close()
    return out


def run_eval(w, params=None, kind="poisson", plan=None, precision="fp32", workspace_limit=0):
    """dlx_eval (fused forward + loss + backward); returns FP64 numpy arrays."""
    from paper_2406_08703_amd import evaluate
    params = params or w.eval_params()
    own = plan is None
    plan = plan or make_plan(w, precision, workspace_limit)
    out = evaluate(plan, dev(params["coeffs"]), dev(params["phase_map"]), dev(params["sources"]),
                   dev(params["flat"]), dev(w.data), kind, w.prior_mu, w.prior_sigma)
    status = plan.sync()
    nz = w.problem.n_zernike
    res = dict(binned=out.binned, model=out.model, loss=out.loss[0], r=out.r, grad_flat=out.grad_flat,
               grad_coeffs=out.grad_zernike[:nz], grad_map=out.grad_map, grad_sources=out.grad_sources)
    res = {k: (None if v is None else v.detach().cpu().numpy().astype(np.float64)) for k, v in res.items()}
    res["loss"] = float(res["loss"])
    res["status"] = status
    if own:
        plan.close()
    return res
