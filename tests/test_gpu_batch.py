"""Many uneven problems in one plan: every problem against the FP64 oracle.

Six problems of the batched configuration at a quarter of its sizes
(pupils 32-128, ragged focal grids such as 63 = 3 x 21, 2-16 wavelengths,
1-3 stars), evaluated in one dlx_eval call over packed arrays, eagerly and
from a captured HIP graph.
"""
import functools

import numpy as np
import pytest

import oracle as O
from synth import make_c4_workloads
from tests.helpers import oracle_problem
from tests.test_gpu_parity import TOL, TOL_BF16X3, compare

pytestmark = pytest.mark.gpu

N_PROBLEMS = 6


@functools.lru_cache(maxsize=None)
def batch():
    items = []
    for w in make_c4_workloads(N_PROBLEMS, scale=0.25):
        prob = oracle_problem(w)
        _, m = O.forward(prob, w.coeffs_true, w.map_true, w.sources_true, w.flat_true)
        w = w.with_data(m)
        p = w.eval_params()
        ref = O.value_and_grad(prob, p["coeffs"], p["phase_map"], p["sources"], p["flat"], w.data, "poisson",
                               w.prior_mu, w.prior_sigma)
        items.append((w, ref))
    return items


def run_batch(precision, graph=False, replays=1, grouped=False):
    import torch
    from paper_2406_08703_amd import BatchPlan
    from tests.gpu_helpers import geometry
    ws = [w for w, _ in batch()]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    bp = BatchPlan([geometry(w) for w in ws], [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws],
                   precision=precision, grouped=grouped)
    assert len(bp.offsets) == len(ws)
    eps = [w.eval_params() for w in ws]
    c = bp.pack("zernike_coeffs", [t(e["coeffs"]) for e in eps])
    s = bp.pack("sources", [t(e["sources"]) for e in eps])
    fl = bp.pack("flat", [t(e["flat"]) for e in eps])
    d = bp.pack("images", [t(w.data) for w in ws])
    out = bp.buffers()
    a = bp.eval_args(c, None, s, fl, d, out, "poisson", ws[0].prior_mu, ws[0].prior_sigma)
    runs = []
    if graph:
        bp.capture(a)
        for _ in range(replays):
            bp.replay()
            torch.cuda.synchronize()
            runs.append({k: (None if v is None else v.clone()) for k, v in out.items()})
    else:
        bp.evaluate(a)
        runs.append(out)
    assert bp.sync() == 0
    res = []
    for run in runs:
        per = []
        views = {n: bp.unpack(f, run[k]) for n, k, f in (
            ("binned", "binned", "images"), ("model", "model", "images"), ("r", "r", "images"),
            ("loss", "loss", "loss"), ("grad_flat", "grad_flat", "flat"),
            ("grad_coeffs", "grad_zernike", "zernike_coeffs"), ("grad_sources", "grad_sources", "sources"))}
        for k in range(len(ws)):
            g = {n: v[k].cpu().numpy().astype(np.float64) for n, v in views.items()}
            g["loss"] = float(g["loss"][0])
            g["grad_map"] = None
            per.append(g)
        res.append(per)
    bp.close()
    return res


@pytest.mark.parametrize("grouped", [False, True])
def test_batch_eval_matches_oracle_per_problem(grouped):
    print(f"batch fp32 eager grouped={grouped}", flush=True)
    got = run_batch("fp32", grouped=grouped)[0]
    for k, (w, ref) in enumerate(batch()):
        P = w.problem
        print(f"problem {k}: Ni={P.n_pupil} No={P.n_focal} Q={P.oversample} nl={len(P.wavelengths)} "
              f"nz={P.n_zernike} ns={P.n_sources}", flush=True)
        compare(got[k], ref, tol_grad=TOL, q=P.oversample)


@pytest.mark.parametrize("grouped", [False, True])
def test_batch_graph_replays_match_eager_bitwise(grouped):
    print(f"batch fp32 graph grouped={grouped}", flush=True)
    eager = run_batch("fp32", grouped=grouped)[0]
    reps = run_batch("fp32", graph=True, replays=3, grouped=grouped)
    for rep in reps:
        for k in range(N_PROBLEMS):
            for n, v in eager[k].items():
                if v is None:
                    continue
                assert np.array_equal(np.asarray(rep[k][n]), np.asarray(v)), (k, n)


@pytest.mark.parametrize("grouped", [False, True])
def test_batch_bf16x3_matches_oracle_per_problem(grouped):
    print(f"batch bf16x3 graph grouped={grouped}", flush=True)
    got = run_batch("bf16x3", graph=True, grouped=grouped)[0]
    for k, (w, ref) in enumerate(batch()):
        compare(got[k], ref, tol_grad=TOL_BF16X3, tol_resid=TOL_BF16X3, tol_img=TOL_BF16X3,
                sources=w.eval_params()["sources"], q=w.problem.oversample, prec="bf16x3")


def test_q1_problem_packed_after_an_odd_sized_problem():
    """A Q = 1 problem whose detector width allows the four-pixel binning kernel, packed after a
    problem with an odd pixel count: its flat and image arrays start at offsets that are not 16-byte
    aligned, so binning takes the one-pixel kernel; both problems must match the oracle."""
    import torch
    from paper_2406_08703_amd import BatchPlan
    from synth import make_workload
    from tests.gpu_helpers import geometry
    print("batch: q1 problem after an odd problem", flush=True)
    ws = [make_workload("c1", n_pupil=24, n_focal=21, oversample=3, noll=tuple(range(2, 8))),
          make_workload("c2", n_pupil=32, n_focal=40, oversample=1, n_wavelengths=3, n_frames=2,
                        noll=tuple(range(2, 9)))]
    assert (ws[0].problem.n_det ** 2) % 4 != 0 and ws[1].problem.n_det % 8 == 0
    refs = []
    for k, w in enumerate(ws):
        prob = oracle_problem(w)
        _, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
        ws[k] = w = w.with_data(m)
        p = w.eval_params()
        refs.append(O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, "poisson",
                                     w.prior_mu, w.prior_sigma))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    bp = BatchPlan([geometry(w) for w in ws], [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws])
    assert bp.offsets[1]["flat"] % 4 != 0 and bp.offsets[1]["images"] % 4 != 0
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
    for k, w in enumerate(ws):
        g = {n: v[k].cpu().numpy().astype(np.float64) for n, v in views.items()}
        g["loss"] = float(g["loss"][0])
        g["grad_map"] = None
        compare(g, refs[k], q=w.problem.oversample)
    bp.close()


@pytest.mark.parametrize("kind", ["poisson", "chi2"])
def test_grouped_launches_with_intrapixel_kernels_match_oracle(kind):
    """With DLX_FLAG_GROUPED one-frame problems run as one launch per stage over all of them; here with a Q x Q
    intra-pixel kernel per problem (packed like the other arrays) and both loss kinds."""
    import dataclasses
    import torch
    from paper_2406_08703_amd import BatchPlan
    from tests.gpu_helpers import geometry
    print(f"grouped launches with intra-pixel kernels, {kind}", flush=True)
    ws, refs = [], []
    for j, w in enumerate(make_c4_workloads(4, scale=0.25)):
        Q = w.problem.oversample
        K = (1.0 + 0.01 * (j + 1) * np.linspace(-1, 1, Q * Q).reshape(Q, Q)).astype(np.float32)
        w = dataclasses.replace(w, intrapixel=K)
        prob = oracle_problem(w)
        _, m = O.forward(prob, w.coeffs_true, None, w.sources_true, w.flat_true)
        w = w.with_data(m)
        p = w.eval_params()
        refs.append(O.value_and_grad(prob, p["coeffs"], None, p["sources"], p["flat"], w.data, kind, w.prior_mu,
                                     w.prior_sigma))
        ws.append(w)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    bp = BatchPlan([geometry(w) for w in ws], [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws],
                   intrapixels=[t(w.intrapixel) for w in ws], grouped=True)
    eps = [w.eval_params() for w in ws]
    c = bp.pack("zernike_coeffs", [t(e["coeffs"]) for e in eps])
    s = bp.pack("sources", [t(e["sources"]) for e in eps])
    fl = bp.pack("flat", [t(e["flat"]) for e in eps])
    d = bp.pack("images", [t(w.data) for w in ws])
    out = bp.buffers()
    a = bp.eval_args(c, None, s, fl, d, out, kind, ws[0].prior_mu, ws[0].prior_sigma)
    bp.capture(a)
    for _ in range(2):
        bp.replay()
    torch.cuda.synchronize()
    assert bp.sync() == 0
    views = {n: bp.unpack(f, out[k]) for n, k, f in (
        ("binned", "binned", "images"), ("model", "model", "images"), ("r", "r", "images"),
        ("loss", "loss", "loss"), ("grad_flat", "grad_flat", "flat"),
        ("grad_coeffs", "grad_zernike", "zernike_coeffs"), ("grad_sources", "grad_sources", "sources"))}
    for k, w in enumerate(ws):
        g = {n: v[k].cpu().numpy().astype(np.float64) for n, v in views.items()}
        g["loss"] = float(g["loss"][0])
        g["grad_map"] = None
        compare(g, refs[k], q=w.problem.oversample, kind=kind)
    bp.close()


def test_grouped_launches_equal_one_plan_per_problem():
    """The batched plan's grouped launches against each problem on a plan of its own: the same
    images bit for bit (the MFT stages' sums do not depend on the tiles), the gradients to rounding."""
    import torch
    from paper_2406_08703_amd import BatchPlan, evaluate
    from tests.gpu_helpers import dev, geometry, make_plan
    from tests.helpers import rel_l2
    print("grouped launches vs one plan per problem", flush=True)
    ws = [w for w, _ in batch()]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    bp = BatchPlan([geometry(w) for w in ws], [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws],
                   grouped=True)
    eps = [w.eval_params() for w in ws]
    out = bp.buffers()
    bp.evaluate(bp.eval_args(bp.pack("zernike_coeffs", [t(e["coeffs"]) for e in eps]), None,
                             bp.pack("sources", [t(e["sources"]) for e in eps]),
                             bp.pack("flat", [t(e["flat"]) for e in eps]), bp.pack("images", [t(w.data) for w in ws]),
                             out, "poisson", ws[0].prior_mu, ws[0].prior_sigma))
    assert bp.sync() == 0
    model = bp.unpack("images", out["model"])
    gz = bp.unpack("zernike_coeffs", out["grad_zernike"])
    gs = bp.unpack("sources", out["grad_sources"])
    for k, (w, e) in enumerate(zip(ws, eps)):
        plan = make_plan(w)
        o = evaluate(plan, dev(e["coeffs"]), None, dev(e["sources"]), dev(e["flat"]), dev(w.data), "poisson",
                     w.prior_mu, w.prior_sigma)
        torch.cuda.synchronize()
        assert torch.equal(o.model, model[k])
        assert rel_l2(gz[k].cpu().numpy(), o.grad_zernike[:w.problem.n_zernike].cpu().numpy()) < 1e-6
        assert rel_l2(gs[k].cpu().numpy(), o.grad_sources.cpu().numpy()) < 1e-6
        plan.close()
    bp.close()
