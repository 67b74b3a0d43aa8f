"""Parity at the full c3 and c5 sizes, in the launch configuration of the benchmark.

The FP64 oracle cannot evaluate every frame at these sizes in a test, so it
evaluates one frame f0 fully (a frame in the last workspace chunk):

* forward: the GPU's binned image and model of frame f0 against the oracle's;
* backward: the gradient is linear in r = dL/dm, so with r equal to the
  oracle's residual on frame f0 and zero on every other frame, the GPU's
  Zernike, map and frame-f0 source gradients must equal the oracle's
  one-frame gradients, and every other frame's source gradients must be
  exactly zero;
* loss: dlx_loss_grad on full-size synthetic model, data and flat against
  the oracle's loss, residual and flat gradient.
"""
import functools

import numpy as np
import pytest

import oracle as O
from synth import make_workload, standin_image
from tests.helpers import oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

FRAME = {"c3": 60, "c5": 15}
TOL = {"fp32": 1e-5, "bf16x3": 1e-4}


@functools.lru_cache(maxsize=None)
def frame_reference(name):
    """Oracle forward, loss and backward of frame f0 of configuration `name`."""
    w = make_workload(name)
    prob = oracle_problem(w)
    f0 = FRAME[name]
    sl = slice(f0, f0 + 1)
    _, m_true = O.forward(prob, w.coeffs_true, w.map_true, w.sources_true[sl], w.flat_true)
    rng = np.random.default_rng(12)
    d0 = rng.poisson(np.clip(m_true, 0, None)).astype(np.float32)
    ep = w.eval_params()
    B, m = O.forward(prob, ep["coeffs"], ep["phase_map"], ep["sources"][sl], ep["flat"])
    L, r, gF, _ = O.loss_grad(m, B, d0, ep["flat"], "poisson", w.prior_mu, w.prior_sigma)
    r32 = r.astype(np.float32)
    gc, gm, gs = O.backward(prob, ep["coeffs"], ep["phase_map"], ep["sources"][sl], ep["flat"], r32)
    return w, dict(binned=B[0], model=m[0], r=r32[0], grad_coeffs=gc, grad_map=gm, grad_sources=gs[0])


@pytest.mark.parametrize("name", ["c3", "c5"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fullsize_frame_forward_and_backward(name, prec):
    import torch
    from tests.gpu_helpers import dev, make_plan
    print(f"full size {name} {prec}", flush=True)
    w, ref = frame_reference(name)
    P = w.problem
    f0 = FRAME[name]
    tol = TOL[prec]
    plan = make_plan(w, precision=prec)
    assert plan.workspace_bytes > 0
    ep = w.eval_params()
    c, pm, s, fl = dev(ep["coeffs"]), dev(ep["phase_map"]), dev(ep["sources"]), dev(ep["flat"])
    B, m = plan.forward(c, pm, s, fl)
    e_b = rel_l2(B[f0].cpu().numpy(), ref["binned"])
    e_m = rel_l2(m[f0].cpu().numpy(), ref["model"])
    r = np.zeros((P.n_frames, P.n_det, P.n_det), np.float32)
    r[f0] = ref["r"]
    gz, gm, gs = plan.backward(c, pm, s, fl, dev(r))
    torch.cuda.synchronize()
    assert plan.sync() == 0
    gs = gs.cpu().numpy()
    errs = dict(binned=e_b, model=e_m, grad_coeffs=rel_l2(gz.cpu().numpy(), ref["grad_coeffs"]),
                grad_pos=rel_l2(gs[f0, :, :2], ref["grad_sources"][:, :2]),
                grad_flux=rel_l2(gs[f0, :, 2], ref["grad_sources"][:, 2]))
    if gm is not None:
        errs["grad_map"] = rel_l2(gm.cpu().numpy(), ref["grad_map"])
    print(" ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    others = np.delete(gs, f0, axis=0)
    assert np.all(others == 0.0)
    plan.close()
    for k, v in errs.items():
        assert v < tol, (k, v)


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_fullsize_loss_matches_oracle(name):
    import torch
    from tests.gpu_helpers import dev, make_plan
    w = make_workload(name)
    P = w.problem
    img = standin_image(w)
    w = w.with_data(img)
    rng = np.random.default_rng(3)
    flat = (w.flat_true * (1 + 0.01 * rng.normal(size=w.flat_true.shape))).astype(np.float32)
    B = (img / w.flat_true[None] * (1 + 0.05 * rng.normal(size=img.shape))).astype(np.float32)
    B = np.abs(B) + 0.5
    m = (flat[None] * B).astype(np.float32)
    plan = make_plan(w)
    L, r, gF = plan.loss_grad(dev(m), dev(B), dev(w.data), dev(flat), "poisson", w.prior_mu, w.prior_sigma)
    torch.cuda.synchronize()
    assert plan.sync() == 0
    Lr, rr, gFr, _ = O.loss_grad(m, B, w.data, flat, "poisson", w.prior_mu, w.prior_sigma)
    plan.close()
    assert abs(float(L.cpu()[0]) - Lr) / abs(Lr) < 1e-12
    assert rel_l2(r.cpu().numpy(), rr) < 1e-7
    assert rel_l2(gF.cpu().numpy(), gFr) < 1e-7
    assert P.n_det ** 2 == gF.numel()


# ------------------------------------------------------------------ the paper's run and the batched configuration
@functools.lru_cache(maxsize=None)
def p0_reference():
    """The paper's run at its full size (integer-dither mode, phase plate), with the benchmark's data."""
    from synth import dithered_standin_image, make_dithered_workload
    w = make_dithered_workload()
    w = w.with_data(dithered_standin_image(w))
    P = w.problem
    big = O.OracleProblem.from_arrays(P.n_pupil, P.n_focal, P.oversample, P.diameter, P.focal_pixel,
                                      P.wavelengths, P.weights, w.transmission, w.zbasis,
                                      phase_screen=w.phase_screen)
    p = w.eval_params()
    ref = O.value_and_grad_dithered(big, p["coeffs"], None, p["sources"], p["flat"], w.data, w.dithers, w.margin,
                                    "poisson", w.prior_mu, w.prior_sigma)
    return w, ref


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fullsize_paper_run_matches_oracle(prec):
    from tests.test_gpu_dither import plan_for, run
    from tests.test_gpu_parity import compare
    print(f"full size p0 {prec}", flush=True)
    w, ref = p0_reference()
    plan = plan_for(w, prec)
    got = run(w, plan, fused=True)     # checks the device status word
    plan.close()
    tol = TOL[prec]
    # the flux gradient sums terms of both signs over all frames: scale by the size of its terms
    rm = np.sum(np.abs(ref["r"] * ref["model"]))
    fscale = rm / np.asarray(w.eval_params()["sources"], np.float64)[:, 2]
    compare(got, ref, tol_grad=tol, tol_resid=tol, tol_img=tol, fscale=fscale)


def test_fullsize_batched_configuration_sampled_problems():
    """All 128 problems of the batched configuration in one plan, as benchmarked; the three cheapest
    problems for the oracle and the largest pupil among the 20 cheapest are checked against it."""
    import torch
    from paper_2406_08703_amd import BatchPlan
    from synth import make_c4_workloads
    from tests.gpu_helpers import geometry
    from tests.test_gpu_parity import compare
    print("full size c4", flush=True)
    ws = [w.with_data(standin_image(w)) for w in make_c4_workloads()]
    cost = [w.problem.n_psf * w.problem.mft_flops() for w in ws]
    order = np.argsort(cost)
    picks = list(order[:3])
    big = max(order[:20], key=lambda k: ws[k].problem.n_pupil)
    if big not in picks:
        picks.append(big)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    bp = BatchPlan([geometry(w) for w in ws], [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws])
    eps = [w.eval_params() for w in ws]
    c = bp.pack("zernike_coeffs", [t(e["coeffs"]) for e in eps])
    s = bp.pack("sources", [t(e["sources"]) for e in eps])
    fl = bp.pack("flat", [t(e["flat"]) for e in eps])
    d = bp.pack("images", [t(w.data) for w in ws])
    out = bp.buffers()
    a = bp.eval_args(c, None, s, fl, d, out, "poisson", ws[0].prior_mu, ws[0].prior_sigma)
    bp.capture(a)
    bp.replay()
    torch.cuda.synchronize()
    assert bp.sync() == 0
    views = {n: bp.unpack(f, out[k]) for n, k, f in (
        ("binned", "binned", "images"), ("model", "model", "images"), ("r", "r", "images"),
        ("loss", "loss", "loss"), ("grad_flat", "grad_flat", "flat"),
        ("grad_coeffs", "grad_zernike", "zernike_coeffs"), ("grad_sources", "grad_sources", "sources"))}
    got_all = {k: {n: v[k].cpu().numpy().astype(np.float64) for n, v in views.items()} for k in picks}
    bp.close()
    for k in picks:
        w = ws[k]
        print(f"problem {k}: pupil {w.problem.n_pupil}, focal {w.problem.n_focal}, {w.problem.n_psf} PSFs",
              flush=True)
        prob = oracle_problem(w)
        e = eps[k]
        ref = O.value_and_grad(prob, e["coeffs"], None, e["sources"], e["flat"], w.data, "poisson", w.prior_mu,
                               w.prior_sigma)
        g = got_all[k]
        g["loss"] = float(g["loss"][0])
        g["grad_map"] = None
        compare(g, ref, sources=e["sources"])
