"""Integer-dither mode (Section 3's run: one enlarged plane, each frame a window of it) on the GPU.

Checked against the FP64 oracle's dithered form (itself pinned to the
per-frame model), against the GPU's own per-frame path with the dithers added
to the star positions, for graph replays and the separate seed pass, and
inside a multi-problem plan next to an ordinary problem.
"""
import dataclasses
import functools

import numpy as np
import pytest

import oracle as O
from synth import make_dithered_workload
from tests.helpers import rel_l2
from tests.test_gpu_parity import TOL, TOL_BF16X3, compare

pytestmark = pytest.mark.gpu

CASES = {
    # Q = 2 with an intra-pixel kernel, 5 frames, windows reaching every edge of the margin
    "q2-k": dict(n_pupil=40, n_det=26, oversample=2, margin=3, n_sources=3, wavelengths=(550e-9, 600e-9, 650e-9),
                 dithers=((0, 0), (3, 3), (3, -3), (-3, 3), (-2, -1)), intra=True),
    # the paper's Q = 1 sampling, ragged sizes
    "q1": dict(n_pupil=36, n_det=37, oversample=1, margin=4, n_sources=4, wavelengths=(545e-9, 595e-9, 645e-9),
               dithers=((0, 0), (4, 4), (4, -4), (-4, 4), (-4, -4)), intra=False),
    # Q = 1 on a 48-pixel enlarged plane (a multiple of 8): the four-pixel binning kernel
    "q1-vec": dict(n_pupil=24, n_det=44, oversample=1, margin=2, n_sources=5, wavelengths=(545e-9, 595e-9, 645e-9),
                   dithers=((0, 0), (2, -2), (-1, 2)), intra=False),
    # more stars than the binning kernel takes at once: 23 stars of 3 wavelengths (21 per pass), and
    # 10 stars of 9 wavelengths (8 per pass, two wavelengths on the first lane)
    "q1-23stars": dict(n_pupil=24, n_det=41, oversample=1, margin=2, n_sources=23,
                       wavelengths=(545e-9, 595e-9, 645e-9), dithers=((0, 0), (2, -2), (-1, 2)), intra=False),
    "q2-10stars-9wl": dict(n_pupil=24, n_det=40, oversample=2, margin=2, n_sources=10,
                           wavelengths=tuple(np.linspace(500e-9, 700e-9, 9)), dithers=((0, 0), (2, 1)), intra=False),
}


@functools.lru_cache(maxsize=None)
def case(name):
    kw = dict(CASES[name])
    intra = kw.pop("intra")
    w = make_dithered_workload(**kw)
    if intra:
        Q = w.problem.oversample
        w = dataclasses.replace(w, intrapixel=(1.0 + 0.004 * np.arange(Q * Q).reshape(Q, Q)).astype(np.float32))
    big = oracle_big(w)
    _, m = O.forward_dithered(big, w.coeffs_true, None, w.sources_true, w.flat_true, w.dithers, w.margin)
    w = w.with_data(m)
    p = w.eval_params()
    ref = O.value_and_grad_dithered(big, p["coeffs"], None, p["sources"], p["flat"], w.data, w.dithers, w.margin,
                                    "poisson", w.prior_mu, w.prior_sigma)
    return w, ref


def oracle_big(w):
    P = w.problem
    return O.OracleProblem.from_arrays(P.n_pupil, P.n_focal, P.oversample, P.diameter, P.focal_pixel,
                                       P.wavelengths, P.weights, w.transmission, w.zbasis, None, w.intrapixel,
                                       w.phase_screen)


def geometry(w, dither=True):
    from paper_2406_08703_amd import Geometry
    P = w.problem
    return Geometry(P.n_pupil, P.oversample * w.n_det, P.oversample, tuple(P.wavelengths), tuple(P.weights),
                    P.n_sources, w.n_frames, P.n_zernike, 0, P.diameter, P.focal_pixel,
                    tuple(map(tuple, w.dithers.tolist())) if dither else (), w.margin if dither else 0)


def plan_for(w, precision="fp32", dither=True, **kw):
    from paper_2406_08703_amd import PsfPlan
    from tests.gpu_helpers import dev
    plan = PsfPlan(geometry(w, dither), dev(w.transmission), dev(w.zbasis), None, dev(w.intrapixel),
                   precision=precision, **kw)
    if w.phase_screen is not None:
        plan.set_phase_screen(dev(w.phase_screen))
    return plan


def to_np(out):
    return {k: (v if isinstance(v, float) or v is None else v.detach().cpu().numpy().astype(np.float64))
            for k, v in out.items()}


def run(w, plan, fused, sources=None):
    from paper_2406_08703_amd import evaluate
    from tests.gpu_helpers import dev
    p = w.eval_params()
    c, s, fl, d = dev(p["coeffs"]), dev(p["sources"] if sources is None else sources), dev(p["flat"]), dev(w.data)
    if fused:
        o = evaluate(plan, c, None, s, fl, d, "poisson", w.prior_mu, w.prior_sigma)
        out = dict(binned=o.binned, model=o.model, loss=float(o.loss[0]), r=o.r, grad_flat=o.grad_flat,
                   grad_coeffs=o.grad_zernike[:w.problem.n_zernike], grad_map=None, grad_sources=o.grad_sources)
    else:
        B, m = plan.forward(c, None, s, fl)
        L, r, gF = plan.loss_grad(m, B, d, fl, "poisson", w.prior_mu, w.prior_sigma)
        gz, _, gs = plan.backward(c, None, s, fl, r)
        out = dict(binned=B, model=m, loss=float(L[0]), r=r, grad_flat=gF, grad_coeffs=gz, grad_map=None,
                   grad_sources=gs)
    assert plan.sync() == 0
    return to_np(out)


@pytest.mark.parametrize("dense", [False, True])
@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("name", list(CASES))
def test_dither_mode_matches_oracle(name, fused, dense):
    # dense: the dense complex MFT products instead of the symmetric fold
    print(f"dither {name} fused={fused} dense={dense}", flush=True)
    w, ref = case(name)
    plan = plan_for(w, dense_mft=dense)
    got = run(w, plan, fused)
    plan.close()
    assert got["grad_sources"].shape == (w.problem.n_sources, 3)
    compare(got, ref, tol_grad=TOL, q=w.problem.oversample)


@pytest.mark.parametrize("name", list(CASES))
def test_dither_mode_bf16x3_matches_oracle(name):
    print(f"dither bf16x3 {name}", flush=True)
    w, ref = case(name)
    plan = plan_for(w, "bf16x3")
    got = run(w, plan, True)
    plan.close()
    # the flux gradient sums terms of both signs over all frames: scale by the size of its terms
    rm = np.sum(np.abs(ref["r"] * ref["model"]))
    fscale = rm / np.asarray(w.eval_params()["sources"], np.float64)[:, 2]
    compare(got, ref, tol_grad=TOL_BF16X3, tol_resid=TOL_BF16X3, tol_img=TOL_BF16X3, fscale=fscale,
            q=w.problem.oversample, prec="bf16x3")


@pytest.mark.parametrize("name", ["q2-k", "q2-10stars-9wl"])
def test_dither_mode_equals_per_frame_path_on_gpu(name):
    # the same frames through the ordinary path, with the dithers added to the positions
    from paper_2406_08703_amd import dlx as C
    print(f"dither vs per-frame {name}", flush=True)
    w, _ = case(name)
    pd = plan_for(w)
    a = run(w, pd, True)
    pd.close()
    pf = plan_for(w, dither=False)
    srcs = w.per_frame_sources(w.eval_params()["sources"])
    b = run(w, pf, True, sources=srcs)
    pf.close()
    if name == "q2-10stars-9wl":
        # one frame per chunk (a 12 MiB workspace holds one of this case's 7.9 MB frames): the fused
        # binning-and-loss launch instead of binning and loss launches over both frames
        p1 = plan_for(w, dither=False, workspace_limit=12 << 20)
        C.dlx_plan_profile(p1.plan, True)
        c1 = run(w, p1, True, sources=srcs)
        launches = C.dlx_plan_stage_times(p1.plan)["BIN"][1]
        C.dlx_plan_profile(p1.plan, False)
        p1.close()
        assert launches == w.n_frames
        for k in ("binned", "model", "r"):
            assert np.array_equal(c1[k], b[k]), k
        # the frame sums and the prior add in another order
        assert rel_l2(c1["grad_flat"], b["grad_flat"]) < 1e-12
        assert abs(c1["loss"] - b["loss"]) <= 1e-12 * abs(b["loss"])
    for k in ("binned", "model", "r", "grad_flat", "grad_coeffs"):
        assert rel_l2(a[k], b[k]) < 1e-5, k
    # to first order the loss moves by sum r dm: an elementwise model error eps (FP32 rounding of the
    # MFT, about 1e-7 here) bounds |dL| by eps sum |r m|
    assert abs(a["loss"] - b["loss"]) < 1e-6 * np.sum(np.abs(b["r"] * b["model"]))
    assert rel_l2(a["grad_sources"], b["grad_sources"].sum(axis=0)) < 1e-5


def test_dither_mode_graph_and_seed_pass_are_bitwise_identical():
    import torch
    from paper_2406_08703_amd import CapturedEval
    from tests.gpu_helpers import dev
    print("dither graph / seed pass", flush=True)
    w, _ = case("q1")
    p = w.eval_params()
    outs = []
    for seed_pass in (False, True):
        plan = plan_for(w, autotune=False, seed_pass=seed_pass)
        outs.append(run(w, plan, True))
        if not seed_pass:
            cap = CapturedEval(plan, dev(p["coeffs"]), None, dev(p["sources"]), dev(p["flat"]), dev(w.data), "poisson",
                               w.prior_mu, w.prior_sigma)
            for _ in range(3):
                o = cap.replay()
                torch.cuda.synchronize()
                assert np.array_equal(o.model.cpu().numpy(), outs[0]["model"].astype(np.float32))
                assert np.array_equal(o.grad_sources.cpu().numpy(), outs[0]["grad_sources"])
        plan.close()
    for k, v in outs[0].items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, outs[1][k]), k


def test_dither_problem_inside_a_multi_problem_plan():
    import torch
    from paper_2406_08703_amd import BatchPlan
    from synth import make_workload
    from tests.gpu_helpers import geometry as plain_geometry
    print("dither in batch", flush=True)
    w, ref = case("q1")
    v = make_workload("c1", n_pupil=24, n_focal=16, noll=tuple(range(2, 8)))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32))
    bp = BatchPlan([plain_geometry(v), geometry(w)], [t(v.transmission), t(w.transmission)], [t(v.zbasis), t(w.zbasis)])
    assert bp.offsets[1]["sources"] == 3 * v.problem.n_frames * v.problem.n_sources
    bp.set_phase_screen(1, t(w.phase_screen).cuda())   # the paper's run carries its phase plate
    pv, pw = v.eval_params(), w.eval_params()
    vd = np.ones((v.problem.n_frames, v.problem.n_det, v.problem.n_det), np.float32) * 3.0
    c = bp.pack("zernike_coeffs", [t(pv["coeffs"]), t(pw["coeffs"])])
    s = bp.pack("sources", [t(pv["sources"]), t(pw["sources"])])
    fl = bp.pack("flat", [t(pv["flat"]), t(pw["flat"])])
    d = bp.pack("images", [t(vd), t(w.data)])
    out = bp.buffers()
    bp.evaluate(bp.eval_args(c, None, s, fl, d, out, "poisson", w.prior_mu, w.prior_sigma))
    assert bp.sync() == 0
    gs = bp.unpack("sources", out["grad_sources"])[1].cpu().numpy()
    loss = float(bp.unpack("loss", out["loss"])[1].cpu()[0])
    bp.close()
    assert rel_l2(gs, ref["grad_sources"]) < TOL
    assert abs(loss - ref["loss"]) < TOL * abs(ref["loss"])


def test_dither_mode_intrapixel_gradient_matches_oracle():
    from paper_2406_08703_amd import evaluate
    from tests.gpu_helpers import dev
    print("dither intrapixel grad", flush=True)
    w, ref = case("q2-k")
    p = w.eval_params()
    want = O.intrapixel_grad_dithered(oracle_big(w), p["coeffs"], None, p["sources"], p["flat"], ref["r"], w.dithers,
                                      w.margin)
    plan = plan_for(w)
    got = evaluate(plan, dev(p["coeffs"]), None, dev(p["sources"]), dev(p["flat"]), dev(w.data), "poisson",
                   w.prior_mu, w.prior_sigma, intrapixel_grad=True).grad_intrapixel.cpu().numpy()
    assert plan.sync() == 0
    plan.close()
    Q = w.problem.oversample
    scale = np.sum(np.abs(np.asarray(p["flat"], np.float64)[None] * ref["r"]) * ref["binned"]) / (Q * Q)
    assert np.max(np.abs(got - want)) / scale < TOL
