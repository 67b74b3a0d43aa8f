"""Static pupil phase screens and Fresnel defocus on the GPU path, against the FP64 oracle.

A binary half-wave plate (the stand-in for the paper's diffractive pupil) is
set on a plan with dlx_plan_set_phase_screen and must give the oracle's
images, loss and gradients through the separate calls, the fused call and a
graph captured before the screen was set; clearing it must give back the
unscreened results bit for bit. A Fresnel defocus enters as one more basis
row; its gradient is that row's entry.
"""
import dataclasses
import functools

import numpy as np
import pytest

import oracle as O
from synth import binary_phase_screen, make_c4_workloads, make_workload
from tests.helpers import oracle_problem
from tests.test_gpu_parity import TOL, compare

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def screened():
    # Q = 3, binary star, sub-pixel dithers, intra-pixel kernel; pupil 80, focal 150 (ragged tiles)
    w = make_workload("c3", n_pupil=80, n_focal=150, n_wavelengths=3, n_frames=2, noll=tuple(range(2, 14)))
    scr = binary_phase_screen(w.problem.n_pupil, np.random.default_rng(11))
    prob = dataclasses.replace(oracle_problem(w), phase_screen=scr.astype(np.float64))
    _, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
    w = w.with_data(m)
    p = w.eval_params()
    ref = O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson", w.prior_mu,
                           w.prior_sigma)
    return w, scr, ref


def test_screened_separate_calls_match_oracle():
    from tests.gpu_helpers import dev, make_plan, run_gpu
    print("screen: separate calls", flush=True)
    w, scr, ref = screened()
    plan = make_plan(w)
    plan.set_phase_screen(dev(scr))
    got = run_gpu(w, plan=plan)
    plan.close()
    assert got["status"] == 0
    compare(got, ref, sources=w.eval_params()["sources"], q=w.problem.oversample)


def test_screened_fused_and_graph_match_oracle_and_clearing_restores_bits():
    import torch
    from paper_2406_08703_amd import CapturedEval
    from tests.gpu_helpers import dev, make_plan, run_eval
    print("screen: fused, graph, clear", flush=True)
    w, scr, ref = screened()
    plan = make_plan(w)
    plain = run_eval(w, plan=plan)
    p = w.eval_params()
    cap = CapturedEval(plan, dev(p["coeffs"]), None, dev(p["sources"]), dev(p["flat"]), dev(w.data), "poisson",
                       w.prior_mu, w.prior_sigma)
    plan.set_phase_screen(dev(scr))          # after the capture: the replay must see it
    fused = run_eval(w, plan=plan)
    assert fused["status"] == 0
    compare(fused, ref, sources=p["sources"], q=w.problem.oversample)
    o = cap.replay()
    torch.cuda.synchronize()
    assert plan.sync() == 0
    assert np.array_equal(o.model.cpu().numpy().astype(np.float64), fused["model"])
    assert np.array_equal(o.grad_zernike[:w.problem.n_zernike].cpu().numpy().astype(np.float64),
                          fused["grad_coeffs"])
    plan.set_phase_screen(None)
    again = run_eval(w, plan=plan)
    for k in ("model", "grad_flat", "grad_coeffs", "grad_sources"):
        assert np.array_equal(again[k], plain[k]), k
    assert again["loss"] == plain["loss"]
    cap = None
    plan.close()


def test_batch_plan_screen_applies_to_its_problem_only():
    import torch
    from paper_2406_08703_amd import BatchPlan
    from tests.gpu_helpers import dev, geometry
    print("screen: batch", flush=True)
    ws, refs, scrs = [], [], []
    for k, w in enumerate(make_c4_workloads(3, scale=0.25)):
        scr = binary_phase_screen(w.problem.n_pupil, np.random.default_rng(20 + k)) if k == 1 else None
        prob = dataclasses.replace(oracle_problem(w), phase_screen=None if scr is None else scr.astype(np.float64))
        _, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
        w = w.with_data(m)
        p = w.eval_params()
        refs.append(O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson",
                                     w.prior_mu, w.prior_sigma))
        ws.append(w)
        scrs.append(scr)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    bp = BatchPlan([geometry(w) for w in ws], [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws])
    bp.set_phase_screen(1, dev(scrs[1]))
    eps = [w.eval_params() for w in ws]
    c = bp.pack("zernike_coeffs", [t(e["coeffs"]) for e in eps])
    s = bp.pack("sources", [t(e["sources"]) for e in eps])
    fl = bp.pack("flat", [t(e["flat"]) for e in eps])
    d = bp.pack("images", [t(w.data) for w in ws])
    out = bp.buffers()
    bp.evaluate(bp.eval_args(c, None, s, fl, d, out, "poisson", ws[0].prior_mu, ws[0].prior_sigma))
    assert bp.sync() == 0
    views = {n: bp.unpack(f, out[k]) for n, k, f in (
        ("binned", "binned", "images"), ("model", "model", "images"), ("r", "r", "images"),
        ("loss", "loss", "loss"), ("grad_flat", "grad_flat", "flat"),
        ("grad_coeffs", "grad_zernike", "zernike_coeffs"), ("grad_sources", "grad_sources", "sources"))}
    for k in range(len(ws)):
        g = {n: v[k].cpu().numpy().astype(np.float64) for n, v in views.items()}
        g["loss"] = float(g["loss"][0])
        g["grad_map"] = None
        compare(g, refs[k], sources=eps[k]["sources"], q=ws[k].problem.oversample)
    from paper_2406_08703_amd import dlx as C
    with pytest.raises(C.DlxError):
        C.dlx_plan_set_phase_screen(bp.plan, 3, None)
    bp.close()


def test_fresnel_defocus_row_matches_oracle_and_its_gradient_is_the_row_entry():
    from synth import fresnel_defocus_basis
    from tests.gpu_helpers import run_eval
    print("fresnel defocus", flush=True)
    w = make_workload("c2", n_pupil=64, n_focal=96, n_wavelengths=3, noll=tuple(range(2, 9)))
    P = w.problem
    B = fresnel_defocus_basis(P.n_pupil, P.diameter, 10.0)
    zb = np.concatenate([w.zbasis, B[None]], axis=0)
    delta_true, delta_eval = 1.5e-3, 0.0
    P2 = dataclasses.replace(P, n_zernike=P.n_zernike + 1, noll=P.noll + (0,))
    w = dataclasses.replace(w, problem=P2, zbasis=zb, coeffs_true=np.append(w.coeffs_true, delta_true),
                            coeffs=np.append(w.coeffs, delta_eval).astype(np.float32))
    prob = oracle_problem(w)
    _, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
    w = w.with_data(m)
    p = w.eval_params()
    ref = O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson", w.prior_mu,
                           w.prior_sigma)
    got = run_eval(w)
    assert got["status"] == 0
    compare(got, ref, sources=p["sources"], q=w.problem.oversample)
    g = ref["grad_coeffs"][-1]
    assert abs(got["grad_coeffs"][-1] - g) <= TOL * np.linalg.norm(ref["grad_coeffs"])
    assert abs(g) > 0   # the defocus moves the loss
