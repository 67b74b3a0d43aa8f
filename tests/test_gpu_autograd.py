"""The torch autograd Function over the hand-written adjoint, against the FP64 oracle.

psf_loss(...) returns L (Section 4's objective); L.backward() runs
dlx_psf_backward and hands each parameter dL/d(parameter) times the
incoming gradient. Here the incoming gradient is 2.5 (the loss is scaled
before backward), so every parameter's .grad must be 2.5 times the oracle's
gradient block, in the parameter's own dtype and shape: this checks the
scaling, the casts and the order of the returned gradients, with the focal
fields recomputed in the backward call and with them stored by the forward.
"""
import numpy as np
import pytest

from tests.helpers import rel_l2
from tests.test_gpu_parity import TOL, max_rel, workload, oracle_eval

pytestmark = pytest.mark.gpu

SCALE = 2.5


def check(name, got, want):
    e_l2, e_max = rel_l2(got, want), max_rel(got, want)
    print(f"{name}: rel_l2={e_l2:.2e} max={e_max:.2e}", flush=True)
    assert e_l2 < TOL and e_max < TOL, (name, e_l2, e_max)


def run_autograd(plan, data, params, has_map, kind, mu, sigma):
    import torch
    from paper_2406_08703_amd import psf_loss
    from tests.gpu_helpers import dev
    c = dev(params["coeffs"]).requires_grad_()
    pm = dev(params["phase_map"]).requires_grad_() if has_map else None
    s = dev(params["sources"]).requires_grad_()
    fl = dev(params["flat"]).requires_grad_()
    L = psf_loss(plan, dev(data), c, pm, s, fl, kind, mu, sigma)
    assert L.dtype == torch.float64 and L.shape == ()
    (SCALE * L).backward()
    torch.cuda.synchronize()
    assert plan.sync() == 0
    for t in (c, s, fl) + ((pm,) if has_map else ()):
        assert t.grad is not None and t.grad.dtype == torch.float32 and t.grad.shape == t.shape
    out = dict(loss=float(L.detach().cpu()), coeffs=c.grad.cpu().numpy(), sources=s.grad.cpu().numpy(),
               flat=fl.grad.cpu().numpy())
    if has_map:
        out["phase_map"] = pm.grad.cpu().numpy()
    return out


@pytest.mark.parametrize("store_fields", [False, True])
@pytest.mark.parametrize("case", ["c3-small", "c5-small"])
def test_autograd_gradients_match_oracle(case, store_fields):
    from paper_2406_08703_amd import PsfPlan
    from tests.gpu_helpers import dev, geometry
    print(f"autograd {case} store_fields={store_fields}", flush=True)
    w, _ = workload(case)
    ref = oracle_eval(case, "eval", "poisson")
    plan = PsfPlan(geometry(w), dev(w.transmission), dev(w.zbasis), dev(w.map_basis), dev(w.intrapixel),
                   store_fields=store_fields)
    has_map = w.problem.n_map > 0
    got = run_autograd(plan, w.data, w.eval_params(), has_map, "poisson", w.prior_mu, w.prior_sigma)
    plan.close()
    assert abs(got["loss"] - ref["loss"]) / abs(ref["loss"]) < TOL
    check("coeffs", got["coeffs"], SCALE * ref["grad_coeffs"])
    check("positions", got["sources"][..., :2], SCALE * ref["grad_sources"][..., :2])
    check("fluxes", got["sources"][..., 2], SCALE * ref["grad_sources"][..., 2])
    check("flat", got["flat"], SCALE * ref["grad_flat"])
    if has_map:
        check("phase_map", got["phase_map"], SCALE * ref["grad_map"])


@pytest.mark.parametrize("store_fields", [False, True])
def test_autograd_integer_dither_mode_matches_oracle(store_fields):
    from tests.test_gpu_dither import case, plan_for
    print(f"autograd integer dithers store_fields={store_fields}", flush=True)
    w, ref = case("q1")
    plan = plan_for(w, store_fields=store_fields)
    got = run_autograd(plan, w.data, w.eval_params(), False, "poisson", w.prior_mu, w.prior_sigma)
    plan.close()
    assert got["sources"].shape == (w.problem.n_sources, 3)
    assert abs(got["loss"] - ref["loss"]) / abs(ref["loss"]) < TOL
    check("coeffs", got["coeffs"], SCALE * ref["grad_coeffs"])
    check("positions", got["sources"][..., :2], SCALE * ref["grad_sources"][..., :2])
    check("fluxes", got["sources"][..., 2], SCALE * ref["grad_sources"][..., 2])
    check("flat", got["flat"], SCALE * ref["grad_flat"])


def test_autograd_chi2_loss_matches_oracle():
    from paper_2406_08703_amd import PsfPlan
    from tests.gpu_helpers import dev, geometry
    w, _ = workload("c3-small")
    ref = oracle_eval("c3-small", "eval", "chi2")
    plan = PsfPlan(geometry(w), dev(w.transmission), dev(w.zbasis), None, dev(w.intrapixel))
    got = run_autograd(plan, w.data, w.eval_params(), False, "chi2", w.prior_mu, w.prior_sigma)
    plan.close()
    assert abs(got["loss"] - ref["loss"]) / abs(ref["loss"]) < TOL
    check("coeffs", got["coeffs"], SCALE * ref["grad_coeffs"])
    check("sources", got["sources"], SCALE * ref["grad_sources"])
    check("flat", got["flat"], SCALE * ref["grad_flat"])
