"""Parity at the full c3 and c5 sizes, in the launch configuration of the benchmark.

The FP64 oracle cannot evaluate every frame at these sizes in a test, so it
evaluates one frame f0 fully (a frame in the last workspace chunk), and the
GPU evaluation is arranged so that every other frame drops out of the
gradient exactly: after a first evaluation, each frame f != f0 gets the
GPU's own model as its data, so that its Poisson residual r = 1 - d/m is
exactly zero there. Then

* the images of frame f0 must equal the oracle's (norm-wise, element-wise
  and pixel by pixel);
* r, the flat-field gradient sum_f r B + prior, the Zernike and map
  gradients and frame f0's source gradients must equal the oracle's
  one-frame evaluation, and every other frame's source gradients must be
  exactly zero;
* the loss minus the other frames' terms m - m ln m (summed on the host in
  FP64 from the GPU's model) must equal the oracle's one-frame loss.

This is run through the three separate calls and through the captured HIP
graph of the fused evaluation that the benchmark times.
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
    """Oracle forward, loss and backward of frame f0 of configuration `name`, and its data."""
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
    gc, gm, gs = O.backward(prob, ep["coeffs"], ep["phase_map"], ep["sources"][sl], ep["flat"], r)
    return w, d0[0], dict(binned=B, model=m, loss=L, r=r, grad_flat=gF, grad_coeffs=gc, grad_map=gm,
                          grad_sources=gs)


def other_frames_loss(model, f0):
    """sum over frames f != f0 of m - m ln m (their data equal their model), FP64."""
    m = np.delete(np.asarray(model, np.float64), f0, axis=0)
    return float(np.sum(m - m * np.log(m)))


def frame_view(f0, nz, binned, model, r, loss, grad_flat, grad_zernike, grad_map, grad_sources):
    """Frame f0 of a full-size GPU evaluation as a one-frame result, checking that the other
    frames are out of the gradient (zero residual and zero source gradients)."""
    to = lambda t: None if t is None else t.detach().cpu().numpy().astype(np.float64)
    m, r, gs = to(model), to(r), to(grad_sources)
    assert np.all(np.delete(r, f0, axis=0) == 0.0)
    assert np.all(np.delete(gs, f0, axis=0) == 0.0)
    sl = slice(f0, f0 + 1)
    return dict(binned=to(binned)[sl], model=m[sl], r=r[sl], loss=float(to(loss)[0]) - other_frames_loss(m, f0),
                grad_flat=to(grad_flat), grad_coeffs=to(grad_zernike)[:nz], grad_map=to(grad_map),
                grad_sources=gs[sl])


@pytest.mark.parametrize("name", ["c3", "c5"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fullsize_separate_calls_frame_matches_oracle(name, prec):
    """dlx_psf_forward, dlx_loss_grad and dlx_psf_backward over every frame (the focal fields
    recomputed in the backward call, one workspace chunk at a time)."""
    import torch
    from tests.gpu_helpers import dev, make_plan
    from tests.test_gpu_parity import compare
    print(f"full size separate calls {name} {prec}", flush=True)
    w, d0, ref = frame_reference(name)
    f0 = FRAME[name]
    plan = make_plan(w, precision=prec)
    assert plan.workspace_bytes > 0
    ep = w.eval_params()
    c, pm, s, fl = dev(ep["coeffs"]), dev(ep["phase_map"]), dev(ep["sources"]), dev(ep["flat"])
    B, m = plan.forward(c, pm, s, fl)
    d = m.clone()
    d[f0] = dev(d0)
    L, r, gF = plan.loss_grad(m, B, d, fl, "poisson", w.prior_mu, w.prior_sigma)
    gz, gm, gs = plan.backward(c, pm, s, fl, r)
    torch.cuda.synchronize()
    assert plan.sync() == 0
    got = frame_view(f0, w.problem.n_zernike, B, m, r, L, gF, gz, gm, gs)
    plan.close()
    tol = TOL[prec]
    compare(got, ref, tol_grad=tol, tol_resid=tol, tol_img=tol, sources=ep["sources"][f0:f0 + 1],
            q=w.problem.oversample, prec=prec)


@pytest.mark.parametrize("name", ["c3", "c5"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fullsize_captured_graph_frame_matches_oracle(name, prec):
    """The benchmarked object: the fused evaluation (forward, loss, seed weights and adjoint per
    workspace chunk, the seed formed in the first adjoint product's loader) captured once into a HIP
    graph and replayed, with the autotuned tiles of the benchmark."""
    import torch
    from paper_2406_08703_amd import CapturedEval
    from tests.gpu_helpers import dev, make_plan
    from tests.test_gpu_parity import compare
    print(f"full size graph {name} {prec}", flush=True)
    w, d0, ref = frame_reference(name)
    P = w.problem
    f0 = FRAME[name]
    plan = make_plan(w, precision=prec)
    ep = w.eval_params()
    c, pm, s, fl = dev(ep["coeffs"]), dev(ep["phase_map"]), dev(ep["sources"]), dev(ep["flat"])
    d = torch.zeros((P.n_frames, P.n_det, P.n_det), dtype=torch.float32, device="cuda")
    d[f0] = dev(d0)
    cap = CapturedEval(plan, c, pm, s, fl, d, "poisson", w.prior_mu, w.prior_sigma)
    o = cap.replay()
    torch.cuda.synchronize()
    first = o.model.clone()
    first[f0] = d[f0]
    d.copy_(first)                  # every other frame's data := its model; the graph reads d in place
    o = cap.replay()
    torch.cuda.synchronize()
    assert plan.sync() == 0
    assert torch.equal(torch.cat([o.model[:f0], o.model[f0 + 1:]]), torch.cat([first[:f0], first[f0 + 1:]]))
    got = frame_view(f0, P.n_zernike, o.binned, o.model, o.r, o.loss, o.grad_flat, o.grad_zernike, o.grad_map,
                     o.grad_sources)
    cap = None
    plan.close()
    tol = TOL[prec]
    compare(got, ref, tol_grad=tol, tol_resid=tol, tol_img=tol, sources=ep["sources"][f0:f0 + 1],
            q=P.oversample, prec=prec)


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
    compare(got, ref, tol_grad=tol, tol_resid=tol, tol_img=tol, fscale=fscale, q=w.problem.oversample, prec=prec)


@functools.lru_cache(maxsize=None)
def c4_reference():
    """The batched configuration's 128 problems; the oracle's evaluation of the three cheapest problems
    and of the largest pupil among the 20 cheapest."""
    from synth import make_c4_workloads
    ws = [w.with_data(standin_image(w)) for w in make_c4_workloads()]
    cost = [w.problem.n_psf * w.problem.mft_flops() for w in ws]
    order = np.argsort(cost)
    picks = list(order[:3])
    big = max(order[:20], key=lambda k: ws[k].problem.n_pupil)
    if big not in picks:
        picks.append(big)
    refs = {}
    for k in picks:
        w, e = ws[k], ws[k].eval_params()
        refs[k] = O.value_and_grad(oracle_problem(w), e["coeffs"], None, e["sources"], e["flat"], w.data, "poisson",
                                   w.prior_mu, w.prior_sigma)
    return ws, refs


@pytest.mark.parametrize("grouped", [False, True])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fullsize_batched_configuration_sampled_problems(prec, grouped):
    """All 128 problems of the batched configuration in one plan, replayed from its graph as
    benchmarked; sampled problems are checked against the oracle."""
    import torch
    from paper_2406_08703_amd import BatchPlan
    from tests.gpu_helpers import geometry
    from tests.test_gpu_parity import compare
    print(f"full size c4 {prec} grouped={grouped}", flush=True)
    ws, refs = c4_reference()
    picks = list(refs)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    bp = BatchPlan([geometry(w) for w in ws], [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws],
                   precision=prec, grouped=grouped)
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
    tol = TOL[prec]
    for k in picks:
        w = ws[k]
        print(f"problem {k}: pupil {w.problem.n_pupil}, focal {w.problem.n_focal}, {w.problem.n_psf} PSFs",
              flush=True)
        g = got_all[k]
        g["loss"] = float(g["loss"][0])
        g["grad_map"] = None
        compare(g, refs[k], tol_grad=tol, tol_resid=tol, tol_img=tol, sources=eps[k]["sources"],
                q=w.problem.oversample, prec=prec)
