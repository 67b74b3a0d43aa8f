"""One intra-pixel kernel per detector pixel (DLX_FLAG_PIXEL_KERNEL) against the FP64 oracle:
images, loss and every gradient block, and dL/dK_p per pixel, through the separate calls and the
fused call, with the frames in one chunk and in one chunk per frame."""
import dataclasses
import functools

import numpy as np
import pytest

import oracle as O
from synth import make_workload
from tests.helpers import oracle_problem, rel_l2
from tests.test_gpu_parity import TOL, compare

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def pixel_case(name):
    # Q = 3 (c3-like: binary, sub-pixel dithers, 3 frames), Q = 4 (odd 31-pixel detector) and Q = 1 on a
    # 40-pixel detector (the four-pixel binning kernel)
    if name == "q3":
        w = make_workload("c3", n_pupil=80, n_focal=150, n_wavelengths=3, n_frames=3, noll=tuple(range(2, 14)))
    elif name == "q1":
        w = make_workload("c2", n_pupil=32, n_focal=40, oversample=1, n_wavelengths=3, noll=tuple(range(2, 9)))
    else:
        w = make_workload("c2", n_pupil=50, n_focal=124, n_wavelengths=4, noll=tuple(range(2, 10)))
    P = w.problem
    n, Q = P.n_det, P.oversample
    rng = np.random.default_rng(29)
    K0 = np.asarray(w.intrapixel) if w.intrapixel is not None else np.ones((Q, Q))
    Kp = (K0[None, None] * (1 + 0.03 * rng.normal(size=(n, n, Q, Q)))).astype(np.float32)
    w = dataclasses.replace(w, intrapixel=Kp)
    prob = oracle_problem(w)
    _, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
    w = w.with_data(m)
    p = w.eval_params()
    ref = O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson", w.prior_mu,
                           w.prior_sigma)
    gK = O.intrapixel_grad(prob, p["coeffs"], None, p["sources"], p["flat"], ref["r"])
    return w, ref, gK


def _plan(w, limit=0):
    from paper_2406_08703_amd import PsfPlan
    from tests.gpu_helpers import dev, geometry
    return PsfPlan(geometry(w), dev(w.transmission), dev(w.zbasis), None, dev(w.intrapixel),
                   workspace_limit=limit, pixel_kernel=True)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("name,chunked", [("q3", False), ("q3", True), ("q4", False), ("q1", False)])
def test_pixel_kernel_matches_oracle(name, chunked, fused):
    import torch
    from paper_2406_08703_amd import evaluate
    from tests.gpu_helpers import dev
    print(f"pixel kernel {name} fused={fused} chunked={chunked}", flush=True)
    w, ref, gK_ref = pixel_case(name)
    P = w.problem
    assert P.n_frames > 1 or not chunked
    plan = _plan(w, 12 << 20 if chunked else 0)   # 12 MiB: one frame per chunk
    p = w.eval_params()
    c, s, fl, d = dev(p["coeffs"]), dev(p["sources"]), dev(p["flat"]), dev(w.data)
    if fused:
        o = evaluate(plan, c, None, s, fl, d, "poisson", w.prior_mu, w.prior_sigma, intrapixel_grad=True)
        got = dict(binned=o.binned, model=o.model, loss=float(o.loss[0]), r=o.r, grad_flat=o.grad_flat,
                   grad_coeffs=o.grad_zernike[:P.n_zernike], grad_sources=o.grad_sources)
        gK = o.grad_intrapixel
    else:
        B, m = plan.forward(c, None, s, fl)
        L, r, gF = plan.loss_grad(m, B, d, fl, "poisson", w.prior_mu, w.prior_sigma)
        gK = torch.empty(plan.k_shape, dtype=torch.float64, device="cuda")
        gz, _, gs = plan.backward(c, None, s, fl, r, grad_intrapixel=gK)
        got = dict(binned=B, model=m, loss=float(L[0]), r=r, grad_flat=gF, grad_coeffs=gz, grad_sources=gs)
    assert plan.sync() == 0
    plan.close()
    got = {k: (v if isinstance(v, float) else v.detach().cpu().numpy().astype(np.float64)) for k, v in got.items()}
    got["grad_map"] = None
    compare(got, ref, sources=p["sources"], q=w.problem.oversample)
    gK = gK.cpu().numpy()
    assert gK.shape == gK_ref.shape
    # dL/dK_p[a,b] sums flat_p r_fp I_f(p,a,b) over frames, terms of both signs; an error eps of the
    # sub-pixel intensities shows up as eps times the size of those terms, sum_f |flat r| B / Q^2
    Q = P.oversample
    flat = np.asarray(w.eval_params()["flat"], np.float64)
    scale = np.sum(np.abs(flat[None] * ref["r"]) * ref["binned"], axis=0) / (Q * Q)
    err = np.max(np.abs(gK - gK_ref)) / np.max(scale)
    print(f"dL/dK_p rel={rel_l2(gK, gK_ref):.2e} cond={err:.2e}", flush=True)
    assert err < TOL
    assert rel_l2(gK, gK_ref) < 10 * TOL


def test_pixel_kernel_is_refused_in_integer_dither_mode():
    from paper_2406_08703_amd import dlx as C
    from tests.test_gpu_dither import case, plan_for
    w, _ = case("q1")
    with pytest.raises(C.DlxError) as e:
        plan_for(w, pixel_kernel=True)
    assert e.value.status == C.DLX_ERR_UNSUPPORTED


@pytest.mark.parametrize("pixel_kernel", [False, True])
def test_batch_plan_intrapixel_gradient_matches_oracle(pixel_kernel):
    """dL/dK through a multi-problem plan: three uneven problems (Q 2 to 4), each with its own
    intra-pixel kernel (one per pixel with pixel_kernel), packed at the plan's offsets."""
    import dataclasses
    import torch
    from paper_2406_08703_amd import BatchPlan
    from synth import make_c4_workloads
    from tests.gpu_helpers import geometry
    print(f"batch dL/dK pixel_kernel={pixel_kernel}", flush=True)
    rng = np.random.default_rng(31)
    ws, refs, gks = [], [], []
    for w in make_c4_workloads(3, scale=0.25):
        P = w.problem
        n, Q = P.n_det, P.oversample
        K = 1.0 + 0.02 * rng.normal(size=(n, n, Q, Q) if pixel_kernel else (Q, Q))
        w = dataclasses.replace(w, intrapixel=K.astype(np.float32))
        prob = oracle_problem(w)
        _, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
        w = w.with_data(m)
        p = w.eval_params()
        ref = O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson", w.prior_mu,
                               w.prior_sigma)
        gks.append(O.intrapixel_grad(prob, p["coeffs"], None, p["sources"], p["flat"], ref["r"]))
        ws.append(w)
        refs.append(ref)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    bp = BatchPlan([geometry(w) for w in ws], [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws],
                   intrapixels=[t(w.intrapixel) for w in ws], pixel_kernel=pixel_kernel)
    eps = [w.eval_params() for w in ws]
    c = bp.pack("zernike_coeffs", [t(e["coeffs"]) for e in eps])
    s = bp.pack("sources", [t(e["sources"]) for e in eps])
    fl = bp.pack("flat", [t(e["flat"]) for e in eps])
    d = bp.pack("images", [t(w.data) for w in ws])
    out = bp.buffers(intrapixel_grad=True)
    bp.evaluate(bp.eval_args(c, None, s, fl, d, out, "poisson", ws[0].prior_mu, ws[0].prior_sigma))
    assert bp.sync() == 0
    gk = bp.unpack("intrapixel", out["grad_intrapixel"])
    models = bp.unpack("images", out["model"])
    for k, w in enumerate(ws):
        assert rel_l2(models[k].cpu().numpy(), refs[k]["model"]) < TOL
        got = gk[k].cpu().numpy()
        Q = w.problem.oversample
        flat = np.asarray(eps[k]["flat"], np.float64)
        scale = np.sum(np.abs(flat[None] * refs[k]["r"]) * refs[k]["binned"]) / (Q * Q)
        if pixel_kernel:
            scale = np.max(np.sum(np.abs(flat[None] * refs[k]["r"]) * refs[k]["binned"], axis=0)) / (Q * Q)
        err = np.max(np.abs(got - gks[k])) / scale
        print(f"problem {k} Q={Q}: dL/dK cond={err:.2e}", flush=True)
        assert got.shape == gks[k].shape
        assert err < TOL
    bp.close()
