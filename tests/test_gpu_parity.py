"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Relative errors are norm-wise per block (per frame for images): the
tolerance 1e-5 for FP32 arithmetic is the target the MFT path is held to.
The flat-field gradient and the loss are reduced in FP64 on the device.
"""
import functools

import numpy as np
import pytest

import oracle as O
from synth import make_workload
from tests.helpers import oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5

CASES = {
    "c1": ("c1", {}),
    "c2": ("c2", {}),
    # binary, intra-pixel kernel, sub-pixel dithers, Q = 3; focal 150 = 96 + 54 (ragged tile)
    "c3-small": ("c3", dict(n_pupil=80, n_focal=150, n_wavelengths=3, n_frames=3, noll=tuple(range(2, 18)))),
    # bicubic map; pupil 100 is not a multiple of 16 (ragged K), focal 136 = 128 + 8
    "c5-small": ("c5", dict(n_pupil=100, n_focal=136, n_wavelengths=2, n_frames=2, noll=tuple(range(2, 22)),
                            n_map=8)),
    # odd detector (31 px), Q = 4
    "c2-odd": ("c2", dict(n_pupil=50, n_focal=124, n_wavelengths=4, noll=tuple(range(2, 10)))),
    # degenerate: no Zernike terms, a 4 x 4 detector
    "tiny-noz": ("c1", dict(n_pupil=16, n_focal=8, noll=())),
    # odd pupil and focal sizes (unpaired middle samples on both sides of the symmetric fold),
    # Q = 3, and the paper's Q = 1 sampling with an obstructed, odd pupil
    "odd-q3": ("c1", dict(n_pupil=33, n_focal=39, oversample=3, noll=tuple(range(2, 12)))),
    "odd-q1": ("c2", dict(n_pupil=31, n_focal=37, oversample=1, n_wavelengths=3, noll=tuple(range(2, 9)))),
    # Q = 1 with a detector width and fold split that are multiples of 4: the four-pixel binning kernel
    "q1-vec": ("c2", dict(n_pupil=32, n_focal=40, oversample=1, n_wavelengths=3, noll=tuple(range(2, 9)))),
    # a 70 x 70 bicubic map: more map columns than the map-gradient kernels take in one pass (64)
    "c5-map70": ("c5", dict(n_pupil=72, n_focal=48, n_wavelengths=1, n_frames=1, noll=tuple(range(2, 8)), n_map=70)),
    # short contractions with many PSFs: every folded depth below one 16-deep k-stage (pupil 24,
    # focal 27), and one full stage plus a partial one holding the unpaired middle term (pupil 40,
    # focal 39); 3 frames x 2 stars x 3 wavelengths
    "k1-groups": ("c3", dict(n_pupil=24, n_focal=27, n_wavelengths=3, n_frames=3, noll=tuple(range(2, 12)))),
    "k2-odd-groups": ("c3", dict(n_pupil=40, n_focal=39, n_wavelengths=3, n_frames=3, noll=tuple(range(2, 12)))),
}


@functools.lru_cache(maxsize=None)
def workload(case):
    name, ov = CASES[case]
    w = make_workload(name, **ov)
    prob = oracle_problem(w)
    B, m = O.forward(prob, w.coeffs_true, w.map_true, w.sources_true, w.flat_true)
    return w.with_data(m), prob


@functools.lru_cache(maxsize=None)
def oracle_eval(case, point, kind):
    w, prob = workload(case)
    p = w.eval_params() if point == "eval" else w.truth_params()
    return O.value_and_grad(prob, p["coeffs"], p["phase_map"], p["sources"], p["flat"], w.data, kind,
                            w.prior_mu, w.prior_sigma)


def flux_scale(want, sources):
    """Per (frame, star) size of the flux gradient's contributions, sum_p |r m| / phi.

    dL/dphi = sum_p r m_s / phi is a sum of terms of both signs that cancel
    ~10x at the evaluation point; an elementwise error eps of the images
    shows up as eps * scale, not eps * |dL/dphi|.
    """
    rm = np.sum(np.abs(want["r"] * want["model"]), axis=(1, 2))
    return rm[:, None] / np.asarray(sources, np.float64)[..., 2]


EPS32 = 2.0 ** -24   # unit roundoff of FP32


def max_rel(a, b):
    """max |a - b| / max |b|: the element-wise half of the relative-error definition."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (nb if nb > 0 else 1.0)) if b.size else 0.0


def pixel_errors(got, want, q, kind="poisson", min_counts=1.0):
    """Per-pixel errors of the images and the residual on the scale the arithmetic sets.

    A pixel sums q^2 focal samples of w phi K F |E|^2 over stars and wavelengths. If every
    focal field E is accurate to eta in max norm (|dE| <= eta max|E|), then
    |d|E|^2| <= 2 eta |E| max|E| + eta^2 max|E|^2, and by Cauchy-Schwarz over the pixel's
    terms |dm_p| <= 2 eta sqrt(m_p X_p) + eta^2 X_p, where X_p = F_p sum w phi K max|E|^2 over
    the pixel's terms is at most about 2 q^2 times the frame's brightest pixel m_max (flat and
    intra-pixel kernel near 1; a 0.3 binary companion peaks elsewhere). So the per-pixel error
    scales as sqrt(m_p m_max), not as m_p: in the faint wings |dm|/m grows like sqrt(m_max/m_p).
    Returned: e_img = max_p |dm_p| / (q sqrt(m_p m_max)) for `binned` and `model` (the field
    accuracy eta up to a factor 3), and e_r = max_p |dr_p| / bound_p for the Poisson residual
    r = 1 - d/m, whose error follows from the model's: dr = (d/m) dm/m, with d/m = 1 - r, plus
    FP32 rounding of the division and subtraction: bound_p = (1 - r_p) 3 q sqrt(m_max/m_p) +
    4 eps (2 - r_p) per unit eta (the caller multiplies by its tolerance). Pixels where the
    oracle's model is below `min_counts` are left out.
    """
    out = {}
    F = want["model"].shape[0]
    for k in ("binned", "model"):
        e = 0.0
        for f in range(F):
            ref = np.asarray(want[k][f], np.float64)
            m = np.asarray(want["model"][f], np.float64)
            sel = m >= min_counts
            if not np.any(sel):
                continue
            mmax = np.max(ref)
            d = np.abs(np.asarray(got[k][f], np.float64) - ref)[sel]
            e = max(e, float(np.max(d / (q * np.sqrt(ref[sel] * mmax)))))
        out[k] = e
    if kind == "poisson":
        worst_scale = 0.0   # max_p |dr_p| measured against the rounding part alone, for the report
        e = 0.0
        for f in range(F):
            m = np.asarray(want["model"][f], np.float64)
            sel = m >= min_counts
            if not np.any(sel):
                continue
            r = np.asarray(want["r"][f], np.float64)[sel]
            dm = (1.0 - r)                                   # d / m
            shape = dm * 3.0 * q * np.sqrt(np.max(m) / m[sel])
            rnd = 4.0 * EPS32 * (2.0 - r)
            dr = np.abs(np.asarray(got["r"][f], np.float64)[sel] - r)
            excess = (dr - rnd).clip(min=0.0)
            # d = 0 gives r = 1 exactly whatever m is (shape 0): any excess there is a failure
            ratio = np.divide(excess, shape, out=np.where(excess > 0, np.inf, 0.0), where=shape > 0)
            e = max(e, float(np.max(ratio)))
            worst_scale = max(worst_scale, float(np.max(dr / np.maximum(np.abs(r), 1.0))))
        out["r"] = e
        out["r_abs_over_max1r"] = worst_scale
    return out


def compare(got, want, tol_grad=TOL, tol_resid=TOL, tol_img=TOL, verbose=True, sources=None, fscale=None, q=1,
            kind="poisson", prec="fp32"):
    """Assert the GPU evaluation `got` equals the oracle's `want` to the given tolerances.

    Every block is held norm-wise (relative L2; images per frame) and element-wise
    (max |d| / max |ref|) to its tolerance, and the images and the Poisson residual pixel by
    pixel to the bound their arithmetic sets (pixel_errors). The flux gradient is held
    norm-wise in FP32; under BF16x3 it is held relative to the size of its terms
    (flux_scale) when `sources` or `fscale` is given.
    """
    errs = {}
    F = want["binned"].shape[0]
    errs["binned"] = max(rel_l2(got["binned"][f], want["binned"][f]) for f in range(F))
    errs["model"] = max(rel_l2(got["model"][f], want["model"][f]) for f in range(F))
    errs["loss"] = abs(got["loss"] - want["loss"]) / abs(want["loss"])
    errs["r"] = rel_l2(got["r"], want["r"])
    errs["grad_flat"] = rel_l2(got["grad_flat"], want["grad_flat"])
    if want["grad_coeffs"].size:
        errs["grad_coeffs"] = rel_l2(got["grad_coeffs"], want["grad_coeffs"])
    errs["grad_pos"] = rel_l2(got["grad_sources"][..., :2], want["grad_sources"][..., :2])
    errs["grad_flux"] = rel_l2(got["grad_sources"][..., 2], want["grad_sources"][..., 2])
    if want["grad_map"] is not None:
        errs["grad_map"] = rel_l2(got["grad_map"], want["grad_map"])
    # element-wise: max |d| / max |ref| per block (images per frame)
    mx = {}
    for k in ("binned", "model"):
        mx[k] = max(max_rel(got[k][f], want[k][f]) for f in range(F))
    mx["r"] = max_rel(got["r"], want["r"])
    mx["grad_flat"] = max_rel(got["grad_flat"], want["grad_flat"])
    if want["grad_coeffs"].size:
        mx["grad_coeffs"] = max_rel(got["grad_coeffs"], want["grad_coeffs"])
    mx["grad_pos"] = max_rel(got["grad_sources"][..., :2], want["grad_sources"][..., :2])
    mx["grad_flux"] = max_rel(got["grad_sources"][..., 2], want["grad_sources"][..., 2])
    if want["grad_map"] is not None:
        mx["grad_map"] = max_rel(got["grad_map"], want["grad_map"])
    pix = pixel_errors(got, want, q, kind)
    for k, v in mx.items():
        errs[k + "_max"] = v
    for k, v in pix.items():
        errs[k + "_pix"] = v
    cond = None
    if fscale is None and sources is not None:
        fscale = flux_scale(want, sources)
    if fscale is not None:
        d = np.abs(got["grad_sources"][..., 2] - want["grad_sources"][..., 2])
        cond = float(np.max(d / fscale))
        errs["grad_flux_cond"] = cond
    if verbose:
        print(" ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k in ("binned", "model", "loss"):
        assert errs[k] < tol_img, (k, errs[k])
    for k in ("r", "grad_flat"):
        assert errs[k] < tol_resid, (k, errs[k])
    for k in ("binned", "model"):
        assert mx[k] < tol_img, (k + "_max", mx[k])
        assert pix[k] < 3.0 * tol_img, (k + "_pix", pix[k])
    for k in ("r", "grad_flat"):
        assert mx[k] < tol_resid, (k + "_max", mx[k])
    if "r" in pix:
        assert pix["r"] < tol_img, ("r_pix", pix["r"])
    flux_by_terms = prec == "bf16x3" and cond is not None
    for k in ("grad_coeffs", "grad_pos", "grad_flux", "grad_map"):
        if k not in errs or (k == "grad_flux" and flux_by_terms):
            continue
        assert errs[k] < tol_grad, (k, errs[k])
        assert mx[k] < tol_grad, (k + "_max", mx[k])
    if flux_by_terms:
        assert cond < tol_grad, ("grad_flux_cond", cond)
    return errs


@pytest.mark.parametrize("case", list(CASES))
def test_forward_loss_gradient_match_oracle(case):
    from tests.gpu_helpers import run_gpu
    print(f"case {case}", flush=True)
    w, _ = workload(case)
    got = run_gpu(w)
    assert got["status"] == 0
    compare(got, oracle_eval(case, "eval", "poisson"), q=w.problem.oversample)


def test_q1_four_pixel_binning_equals_one_pixel_binning():
    # the separate forward call bins four pixels per thread at this size; the fused evaluation (one
    # frame per chunk) bins one pixel per thread together with the loss: the same bits
    from tests.gpu_helpers import run_eval, run_gpu
    w, _ = workload("q1-vec")
    assert w.problem.oversample == 1 and w.problem.n_det % 8 == 0
    a, b = run_gpu(w), run_eval(w)
    for k in ("binned", "model"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("case", ["c3-small", "c5-small", "c2", "odd-q3"])
def test_binning_kernels_agree_bitwise_at_every_compiled_oversampling(case):
    # the separate forward call bins every frame of a chunk in one launch (intensity_kernel); a fused
    # evaluation with one frame per chunk bins together with the loss (bin_loss_kernel). Q = 3
    # (c3-small, odd-q3), 2 (c5-small) and 4 (c2) each have their own compiled path: the same bits
    from paper_2406_08703_amd.dlx import DlxError
    from tests.gpu_helpers import make_plan, run_eval, run_gpu
    w, _ = workload(case)
    # the smallest workspace limit a plan accepts holds one frame per chunk
    full = make_plan(w, autotune=False)
    lo, hi = 1 << 16, full.workspace_bytes
    full.close()
    while hi - lo > 4096:
        mid = (lo + hi) // 2
        try:
            make_plan(w, workspace_limit=mid, autotune=False).close()
            hi = mid
        except DlxError:
            lo = mid
    plan = make_plan(w, workspace_limit=hi)
    a, b = run_gpu(w, plan=plan), run_eval(w, plan=plan)
    plan.close()
    for k in ("binned", "model"):
        assert np.array_equal(a[k], b[k]), k


def test_chi2_variant_matches_oracle():
    from tests.gpu_helpers import run_gpu
    w, _ = workload("c3-small")
    got = run_gpu(w, kind="chi2")
    compare(got, oracle_eval("c3-small", "eval", "chi2"), q=w.problem.oversample, kind="chi2")


def test_truth_point_c2():
    # At the truth r = 1 - d/m is photon noise, ~1/sqrt(m) per pixel, and every gradient
    # block is a sum of terms that cancel to that noise level. An FP32 model error eps
    # (~1e-7 here) enters r as eps * d/m ~ eps and the blocks relative to their small
    # values as ~eps * sqrt(m_peak) (peak counts ~1e6 at 1e8 photons): about 1e-4. The
    # images and the loss are not affected and keep the 1e-5 bar.
    from tests.gpu_helpers import run_gpu
    w, _ = workload("c2")
    got = run_gpu(w, params=w.truth_params())
    errs = compare(got, oracle_eval("c2", "truth", "poisson"), tol_grad=2e-3, tol_resid=2e-4, q=w.problem.oversample)
    print("truth-point errors", errs)


def test_replays_are_bitwise_identical():
    from tests.gpu_helpers import make_plan, run_gpu
    w, _ = workload("c3-small")
    plan = make_plan(w)
    a = run_gpu(w, plan=plan)
    b = run_gpu(w, plan=plan)
    plan.close()
    for k in ("binned", "model", "r", "grad_flat", "grad_coeffs", "grad_sources"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["loss"] == b["loss"]


def test_frame_chunking_gives_same_results():
    from tests.gpu_helpers import make_plan, run_gpu
    w, _ = workload("c3-small")
    one = run_gpu(w)
    small = make_plan(w, workspace_limit=12 << 20)   # forces one frame per chunk
    got = run_gpu(w, plan=small)
    small.close()
    np.testing.assert_array_equal(got["binned"], one["binned"])
    assert rel_l2(got["grad_coeffs"], one["grad_coeffs"]) < 1e-6
    compare(got, oracle_eval("c3-small", "eval", "poisson"), q=w.problem.oversample)


def test_status_word_reports_domain_and_nonfinite():
    import torch
    from tests.gpu_helpers import make_plan, dev
    w, _ = workload("c1")
    plan = make_plan(w)
    shp = (1, w.problem.n_det, w.problem.n_det)
    m = torch.ones(shp, device="cuda")
    B = torch.ones(shp, device="cuda")
    d = torch.ones(shp, device="cuda")
    fl = dev(w.flat)
    m[0, 3, 4] = 0.0
    plan.loss_grad(m, B, d, fl)
    assert plan.sync() == 6   # DLX_ERR_DOMAIN
    assert plan.sync() == 0   # cleared
    m[0, 3, 4] = 1.0
    d[0, 1, 1] = float("nan")
    plan.loss_grad(m, B, d, fl)
    assert plan.sync() == 5   # DLX_ERR_NONFINITE
    plan.close()


@pytest.mark.parametrize("case", ["c1", "c2", "c3-small", "c5-small", "c2-odd", "tiny-noz"])
def test_fused_eval_matches_oracle(case):
    # dlx_eval: forward, loss and adjoint per frame chunk, E reused (no recompute)
    from tests.gpu_helpers import run_eval
    print(f"case {case}", flush=True)
    w, _ = workload(case)
    got = run_eval(w)
    assert got["status"] == 0
    compare(got, oracle_eval(case, "eval", "poisson"), q=w.problem.oversample)


def test_fused_eval_chunked_and_chi2():
    from tests.gpu_helpers import run_eval
    w, _ = workload("c3-small")
    got = run_eval(w, workspace_limit=12 << 20)   # one frame per chunk
    compare(got, oracle_eval("c3-small", "eval", "poisson"), q=w.problem.oversample)
    got = run_eval(w, kind="chi2", workspace_limit=12 << 20)
    compare(got, oracle_eval("c3-small", "eval", "chi2"), q=w.problem.oversample, kind="chi2")


def test_graph_replays_match_eager_eval():
    # one captured evaluation replayed several times, with eager work and
    # synchronisations in between; every replay must equal the eager dlx_eval
    import torch
    from paper_2406_08703_amd import CapturedEval, evaluate
    from tests.gpu_helpers import make_plan, dev, run_gpu, run_eval
    w, _ = workload("c3-small")
    plan = make_plan(w, workspace_limit=24 << 20)   # two chunks
    eager = run_eval(w, plan=plan)
    p = w.eval_params()
    c, s, fl, d = dev(p["coeffs"]), dev(p["sources"]), dev(p["flat"]), dev(w.data)
    g = CapturedEval(plan, c, None, s, fl, d, "poisson", w.prior_mu, w.prior_sigma)
    nz = w.problem.n_zernike
    for i in range(4):
        out = g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.model.cpu().numpy(), eager["model"])
        np.testing.assert_array_equal(out.r.cpu().numpy(), eager["r"])
        np.testing.assert_array_equal(out.grad_flat.cpu().numpy(), eager["grad_flat"])
        np.testing.assert_array_equal(out.grad_zernike.cpu().numpy()[:nz], eager["grad_coeffs"])
        np.testing.assert_array_equal(out.grad_sources.cpu().numpy(), eager["grad_sources"])
        assert float(out.loss.cpu()[0]) == eager["loss"]
        run_gpu(w, plan=plan)     # eager work on the same plan between replays
    # inputs updated in place are seen by the next replay
    fl.add_(0.01)
    out = g.replay()
    ref = run_eval(w, plan=plan, params=dict(p, flat=p["flat"] + np.float32(0.01)))
    np.testing.assert_array_equal(out.model.cpu().numpy(), ref["model"])
    np.testing.assert_array_equal(out.grad_zernike.cpu().numpy()[:nz], ref["grad_coeffs"])
    plan.close()


TOL_BF16X3 = 1e-4


@pytest.mark.parametrize("case", ["c1", "c2", "c3-small", "c5-small", "c2-odd", "tiny-noz"])
def test_bf16x3_eval_matches_oracle(case):
    # split-precision MFTs (bf16 hi/lo operands, 3 products, FP32 accumulation)
    from tests.gpu_helpers import run_eval
    print(f"case {case} bf16x3", flush=True)
    w, _ = workload(case)
    got = run_eval(w, precision="bf16x3")
    assert got["status"] == 0
    compare(got, oracle_eval(case, "eval", "poisson"), tol_grad=TOL_BF16X3, tol_resid=TOL_BF16X3,
            tol_img=TOL_BF16X3, sources=w.eval_params()["sources"], q=w.problem.oversample, prec="bf16x3")


def test_bf16x3_standalone_calls_and_chunking():
    from tests.gpu_helpers import make_plan, run_gpu
    w, _ = workload("c3-small")
    plan = make_plan(w, precision="bf16x3", workspace_limit=12 << 20)
    got = run_gpu(w, plan=plan)
    plan.close()
    compare(got, oracle_eval("c3-small", "eval", "poisson"), tol_grad=TOL_BF16X3, tol_resid=TOL_BF16X3,
            tol_img=TOL_BF16X3, sources=w.eval_params()["sources"], q=w.problem.oversample, prec="bf16x3")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["c3-small", "c2-odd"])
def test_separate_seed_pass_is_bitwise_identical(case, prec):
    """The adjoint seed formed by its own pass (the large-frame path) or in B3's loader: same bits."""
    from tests.gpu_helpers import make_plan, run_eval
    print(f"seed pass {case} {prec}", flush=True)
    w, _ = workload(case)
    outs = []
    for seed_pass in (False, True):
        plan = make_plan(w, prec, autotune=False, seed_pass=seed_pass)
        outs.append(run_eval(w, plan=plan))
        plan.close()
    for k, v in outs[0].items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, outs[1][k]), k
        else:
            assert v == outs[1][k], k


def _kgrad_scale(w, ref):
    """Per-entry size of the terms of dL/dK: sum_f sum_p |flat r| I (I from the oracle's binned image)."""
    Q = w.problem.oversample
    return np.sum(np.abs(np.asarray(w.eval_params()["flat"], np.float64)[None] * ref["r"]) * ref["binned"]) / (Q * Q)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("case", ["c3-small", "c2-odd", "c1"])
def test_intrapixel_gradient_matches_oracle(case, fused):
    import torch
    from paper_2406_08703_amd import evaluate
    from tests.gpu_helpers import dev, make_plan
    print(f"intrapixel grad {case} fused={fused}", flush=True)
    w, prob = workload(case)
    ref = oracle_eval(case, "eval", "poisson")
    p = w.eval_params()
    want = O.intrapixel_grad(prob, p["coeffs"], p["phase_map"], p["sources"], p["flat"], ref["r"])
    plan = make_plan(w, workspace_limit=0)
    c, pm, s, fl, d = dev(p["coeffs"]), dev(p["phase_map"]), dev(p["sources"]), dev(p["flat"]), dev(w.data)
    if fused:
        got = evaluate(plan, c, pm, s, fl, d, "poisson", w.prior_mu, w.prior_sigma, intrapixel_grad=True).grad_intrapixel
    else:
        B, m = plan.forward(c, pm, s, fl)
        L, r, gF = plan.loss_grad(m, B, d, fl, "poisson", w.prior_mu, w.prior_sigma)
        Q = w.problem.oversample
        got = torch.empty((Q, Q), dtype=torch.float64, device="cuda")
        plan.backward(c, pm, s, fl, r, grad_intrapixel=got)
    assert plan.sync() == 0
    plan.close()
    got = got.cpu().numpy()
    err = np.max(np.abs(got - want)) / _kgrad_scale(w, ref)
    print(f"dL/dK rel={rel_l2(got, want):.2e} cond={err:.2e}", flush=True)
    assert err < TOL


def test_intrapixel_gradient_rejects_large_oversampling():
    import torch
    from paper_2406_08703_amd import dlx as C
    from tests.gpu_helpers import dev, make_plan
    w = make_workload("c1", n_pupil=16, n_focal=10, oversample=5, noll=())
    plan = make_plan(w)
    P = w.problem
    p = w.eval_params()
    gk = torch.empty((5, 5), dtype=torch.float64, device="cuda")
    r = torch.zeros((P.n_frames, P.n_det, P.n_det), dtype=torch.float32, device="cuda")
    with pytest.raises(C.DlxError) as e:
        plan.backward(None, None, dev(p["sources"]), dev(p["flat"]), r, grad_intrapixel=gk)
    assert e.value.status == C.DLX_ERR_UNSUPPORTED
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["c3-small", "c5-small", "c2-odd", "tiny-noz", "odd-q3", "odd-q1"])
def test_dense_and_folded_mft_agree_with_the_oracle(case, prec):
    """The dense complex products (DLX_FLAG_DENSE_MFT) and the symmetric fold (default) compute the
    same evaluation: each matches the oracle, and the two agree to rounding. The cases cover odd and
    even pupil and focal sizes (unpaired middle samples), ragged tiles and padded rows."""
    from tests.gpu_helpers import make_plan, run_eval, run_gpu
    print(f"dense vs fold {case} {prec}", flush=True)
    w, _ = workload(case)
    ref = oracle_eval(case, "eval", "poisson")
    tol = TOL if prec == "fp32" else TOL_BF16X3
    outs = {}
    for dense in (False, True):
        plan = make_plan(w, prec, dense_mft=dense)
        got = run_eval(w, plan=plan)
        sep = run_gpu(w, plan=plan)
        plan.close()
        assert got["status"] == 0 and sep["status"] == 0
        kw = dict(tol_grad=tol, tol_resid=tol, tol_img=tol, sources=w.eval_params()["sources"],
                  q=w.problem.oversample, prec=prec)
        compare(got, ref, **kw)
        compare(sep, ref, **kw)
        outs[dense] = got
    assert rel_l2(outs[False]["model"], outs[True]["model"]) < tol
    assert rel_l2(outs[False]["grad_coeffs"], outs[True]["grad_coeffs"]) < 10 * tol


# Tiles, B4's K split and its PSFs per group forced through the tune cache (whatever the tuner would
# pick): a 4-way split leaves splits with no k-stage at these depths, and one B4 group holding every
# PSF makes each B4 workgroup run its tile stream through all of them, the next PSF's first tiles
# stored and fetched during the last stages of the one before (one stage per PSF at k1-groups).
FORCED = [  # F1, F2, B3, B4 tiles (32 WM x 32 WN), B4 K split
    ((1, 1), (1, 1), (1, 1), (1, 1), 4),
    ((2, 2), (2, 2), (2, 2), (2, 2), 2),
    ((2, 1), (1, 2), (2, 1), (2, 1), 1),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["k1-groups", "k2-odd-groups"])
def test_forced_tiles_splits_and_groups_match_oracle(case, prec, tmp_path, monkeypatch):
    from tests.gpu_helpers import make_plan, run_eval
    print(f"forced tiles {case} {prec}", flush=True)
    w, _ = workload(case)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("DLX_TUNE_CACHE", str(path))
    make_plan(w, prec).close()   # tunes and writes the shape's line
    key = path.read_text().splitlines()[0].split(" : ")[0]
    P = w.problem
    n_psf = P.n_frames * P.n_sources * len(P.wavelengths)
    want = oracle_eval(case, "eval", "poisson")
    kw = dict(q=P.oversample) if prec == "fp32" else dict(
        tol_grad=TOL_BF16X3, tol_resid=TOL_BF16X3, tol_img=TOL_BF16X3, sources=w.eval_params()["sources"],
        q=P.oversample, prec="bf16x3")
    for f1, f2, b3, b4, ks in FORCED:
        vals = [*f1, *f2, *b3, *b4, ks, n_psf]
        path.write_text(f"{key} : {' '.join(map(str, vals))}\n")
        plan = make_plan(w, prec)
        assert plan.tiles == {"F1": (32 * f1[0], 32 * f1[1]), "F2": (32 * f2[0], 32 * f2[1]),
                              "B3": (32 * b3[0], 32 * b3[1]), "B4": (32 * b4[0], 32 * b4[1])}
        got = run_eval(w, plan=plan)
        plan.close()
        assert got["status"] == 0
        print(f"  tiles {vals}", flush=True)
        compare(got, want, **kw)
