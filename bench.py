"""Forward + gradient throughput of the differentiable PSF path on one MI355X.

One step = one value-and-gradient evaluation (forward model, loss, adjoint)
over the whole workload -- every wavelength, star and frame -- replayed from
the captured HIP graph, inputs resident in HBM. The default workload is c3
(4,096 PSFs of 512 -> 768 per step) in FP32, with a BF16x3 record of the
same evaluation beside it. Prints one JSON line: PSF evals/s, MFT TFLOP/s,
the roofline of the dominant MFT stage (timed with HIP events on its
stream), the FP64 oracle's throughput on one full frame on the host cores,
and the relative errors of that frame's evaluation against the oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c3] [--precision fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0   # dense
HBM_PEAK_GBS = 8000.0
METRIC = "fwd+grad PSF evals/s & MFT TFLOP/s (% MFMA peak) at rel err ≤1e-5 vs FP64"

WORKLOADS = {
    "c1": "64x64 pupil -> 64x64 focal (Q=2, 32x32 det), 1 wavelength, 1 star, 1 frame, 10 Zernikes",
    "c2": "256x256 obstructed pupil -> 512x512 focal (Q=4, 128x128 det), 20 wavelengths 500-700 nm, "
          "1 star, 1 frame, 64 Zernikes, 16384 flat-field pixels",
    "c3": "512x512 pupil -> 768x768 focal (Q=3, 256x256 det), 32 wavelengths, binary star, 64 dithered "
          "frames, 128 Zernikes, intra-pixel kernel",
    "c5": "1024x1024 pupil -> 2048x2048 focal (Q=2, 1024x1024 det), 16 wavelengths, 1 star, 16 dithered "
          "frames, 256 Zernikes + 64x64 bicubic map",
    "c4": "128 independent uneven problems in one plan: pupils 128-512, focal 63-256 (Q 2-4), 8-64 "
          "wavelengths 450-800 nm, 16-128 Zernikes, 1-3 stars, 1 frame each",
    "p0": "the paper's run: 512x512 pupil (obstruction radius D/10) with a binary half-wave phase plate (stand-in), "
          "20 stars, 3 wavelengths 545/595/645 nm, 7 Zernikes (Noll 4-10), 1024x1024 detector of 12 mas pixels, 5 frames dithered by (+-20, +-20) px, "
          "integer-dither mode on a 1064x1064 plane",
}


def measured_traffic(config, precision, stage, tile, fold=True):
    """HBM bytes per launch of `stage`'s kernel at `tile` (WM, WN) from the committed rocprofv3 summary.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same
    counters read for a plain copy kernel of known size. Returns None when no
    summary exists, when it lacks this kernel, or when the GEMM source
    changed since it was taken.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{config}_{precision}.txt")
    src = os.path.join(ROOT, "paper_2406_08703_amd", "csrc", "mft_gemm.hip")
    if not os.path.exists(path):
        return None
    fields, stages = {}, {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and parts[0] in ("fetch_scale", "write_scale", "kernel_source_sha256"):
            fields[parts[0]] = parts[1]
        elif len(parts) == 6 and parts[0] == "stage":
            stages[parts[2]] = (float(parts[4]), float(parts[5]))
    if fields.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    kind = {"F1": 0, "F2": 1, "B3": 3, "B4": 4}[stage]
    name = f"{kernel_name(fold)}<{kind},{tile[0]},{tile[1]},{0 if precision == 'fp32' else 1}>"
    if name not in stages:
        return None
    f, w = stages[name]
    return round(1024.0 * (f * float(fields["fetch_scale"]) + w * float(fields["write_scale"])))


def timed_steps(torch, fn, k):
    """Wall time of k steps between two device synchronisations, and each step's device time
    from HIP events recorded on the current stream between the steps."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(k):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [ev[i].elapsed_time(ev[i + 1]) for i in range(k)]


def step_stats(per):
    import statistics
    return {"median": round(statistics.median(per), 5), "min": round(min(per), 5), "max": round(max(per), 5)}


def stage_bytes(P, stage):
    """Algorithmic HBM bytes per evaluation of the memory-bound stages of dlx_eval (each array
    read or written once; FP32 unless noted)."""
    ni, no, nd, F, S, L = P.n_pupil, P.n_focal, P.n_det, P.n_frames, P.n_sources, P.n_wavelengths
    nz, nmap, npsf = P.n_zernike, P.n_map, P.n_psf
    return {
        # OPD (Z, A read), pupil field P0 per wavelength (planar complex), tilt vectors per PSF
        "PREP": 4.0 * (nz + 1) * ni * ni + 8.0 * L * ni * ni + 16.0 * npsf * ni + 4.0 * nmap * ni,
        # E read once; per-star binned images, binned and model written
        "BIN": 8.0 * npsf * no * no + 4.0 * F * (S + 2) * nd * nd,
        # model, binned, data, per-star binned read; r written; seed weights G written
        "LOSS": 4.0 * F * (4 + S) * nd * nd + 4.0 * F * no * no + 12.0 * nd * nd,
        # Zernike basis re-read for the projection, dL/dOPD (FP64) written and read
        "GRAD": 4.0 * nz * ni * ni + 16.0 * ni * ni,
    }.get(stage)


def kernel_name(fold):
    return "fgemm_kernel" if fold else "cgemm_kernel"


def hbm_bytes(P, stage, table):
    """stage_bytes of a timed stage; the fused evaluation bins and forms the loss in one launch
    (stage BIN, no LOSS stage), which then moves the bytes of both."""
    b = stage_bytes(P, stage)
    if stage == "BIN" and "LOSS" not in table:
        b += stage_bytes(P, "LOSS")
    return b


def gemm_roofline(P, gemm, tiles, precision, config, fold=True):
    """Roofline entry of the dominant MFT stage from its HIP-event launch times."""
    dom = max(gemm, key=lambda k: gemm[k]["ms_per_step"])
    dv = gemm[dom]
    flops_per_launch = stage_flops(P, dom, fold) * dv["psfs"] / dv["launches"]
    achieved = flops_per_launch / (dv["avg_launch_ms"] * 1e-3) / 1e12
    tile = tiles[dom]
    kname = (f"{kernel_name(fold)}<{dict(F1=0, F2=1, B3=3, B4=4)[dom]}, {tile[0] // 32}, {tile[1] // 32}, "
             f"{0 if precision == 'fp32' else 1}> ({dom})")
    if precision == "fp32":
        roofline = {"bound": "mfma", "kernel": kname, "achieved": round(achieved, 3),
                    "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4),
                    "traffic": None, "flops_per_launch": flops_per_launch,
                    "avg_launch_ms": round(dv["avg_launch_ms"], 5)}
    else:
        # each real product runs as three BF16 MFMA products (hi*hi + hi*lo + lo*hi)
        bf = 3.0 * achieved
        roofline = {"bound": "mfma", "kernel": kname + " bf16x3", "achieved": round(bf, 3),
                    "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(bf / BF16_MFMA_PEAK_TFLOPS, 4),
                    "traffic": None, "flops_per_launch": 3.0 * flops_per_launch,
                    "avg_launch_ms": round(dv["avg_launch_ms"], 5), "fp32_equivalent_tflops": round(achieved, 3),
                    "frac_of_fp32_mfma_peak": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4)}
    roofline["traffic"] = measured_traffic(config, precision, dom, (tile[0] // 32, tile[1] // 32), fold)
    return roofline


def stage_flops(P, stage, fold=True):
    """Real flops one PSF's product of `stage` executes on the matrix cores (a complex
    multiply-add is four real ones). Dense: the full complex product. Folded: four real
    products over half the DFT rows and half the depth, h = ceil(N / 2)."""
    ni, no = P.n_pupil, P.n_focal
    if not fold:
        return {"F1": 8.0 * no * ni * ni, "F2": 8.0 * no * no * ni,
                "B3": 8.0 * ni * no * no, "B4": 8.0 * ni * ni * no}.get(stage)
    hi, ho = (ni + 1) // 2, (no + 1) // 2
    return {"F1": 8.0 * ho * ni * hi, "F2": 8.0 * no * ho * hi,
            "B3": 8.0 * hi * no * ho, "B4": 8.0 * hi * ni * ho}.get(stage)


def mft_executed_flops(P, fold=True):
    """Flops one PSF's forward + adjoint MFT executes (the four stages)."""
    return sum(stage_flops(P, k, fold) for k in ("F1", "F2", "B3", "B4"))


def frame_index(P):
    """The frame whose oracle evaluation checks a run: one in the last workspace chunk of the
    large configurations (c3: 60 of 64, c5: 15 of 16), the only frame otherwise."""
    F = P.n_frames
    return F - 4 if F >= 8 else F - 1


def block_errors(got, ref, tol, precision):
    """Relative errors of one frame's evaluation against the oracle's, per block: norm-wise
    (relative L2) and element-wise (max |d| / max |ref|). The flux gradient sums terms of both
    signs; under BF16x3 it is also measured against the size of its terms, sum_p |r m| / phi."""
    import numpy as np
    l2 = lambda a, b: float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))
    mx = lambda a, b: float(np.max(np.abs(np.ravel(a) - np.ravel(b))) / max(np.max(np.abs(np.ravel(b))), 1e-300))
    pairs = {"model": (got["model"], ref["model"]), "r": (got["r"], ref["r"]),
             "grad_flat": (got["grad_flat"], ref["grad_flat"]),
             "grad_zernike": (got["grad_coeffs"], ref["grad_coeffs"]),
             "grad_position": (got["grad_sources"][..., :2], ref["grad_sources"][..., :2]),
             "grad_flux": (got["grad_sources"][..., 2], ref["grad_sources"][..., 2])}
    if ref.get("grad_map") is not None:
        pairs["grad_map"] = (got["grad_map"], ref["grad_map"])
    errs = {"loss": abs(got["loss"] - ref["loss"]) / abs(ref["loss"])}
    for k, (x, y) in pairs.items():
        errs[k] = l2(x, y)
        errs[k + "_max"] = mx(x, y)
    flux_terms = np.sum(np.abs(ref["r"] * ref["model"])) / np.asarray(got["phi"], np.float64)
    errs["grad_flux_by_terms"] = float(np.max(np.abs(got["grad_sources"][..., 2] - ref["grad_sources"][..., 2])
                                              / flux_terms))
    held = [v for k, v in errs.items() if not k.startswith("grad_flux")]
    held += [errs["grad_flux_by_terms"]] if precision == "bf16x3" else [errs["grad_flux"], errs["grad_flux_max"]]
    out = {k: float(f"{v:.3e}") for k, v in errs.items()}
    out["max_held"] = float(f"{max(held):.3e}")
    out["tolerance"] = tol
    out["within_tolerance"] = bool(max(held) <= tol)
    return out


def frame_result(cap, d, d_f0, f0, nz):
    """Frame f0 of a full evaluation replayed from `cap`, with every other frame's data set to the
    GPU's own model so that its residual, and its share of every gradient, is exactly zero.
    The loss of frame f0 is the total minus the other frames' terms m - m ln m (FP64 on the host)."""
    import numpy as np
    import torch
    first = cap.out.model.clone()     # the model does not depend on the data
    first[f0] = d_f0
    d.copy_(first)
    o = cap.replay()
    torch.cuda.synchronize()
    to = lambda t: None if t is None else t.detach().cpu().numpy().astype(np.float64)
    m, r, gs = to(o.model), to(o.r), to(o.grad_sources)
    others_zero = bool(np.all(np.delete(r, f0, axis=0) == 0.0) and np.all(np.delete(gs, f0, axis=0) == 0.0))
    mo = np.delete(m, f0, axis=0)
    sl = slice(f0, f0 + 1)
    return dict(model=m[sl], r=r[sl], loss=float(to(o.loss)[0]) - float(np.sum(mo - mo * np.log(mo))),
                grad_flat=to(o.grad_flat), grad_coeffs=to(o.grad_zernike)[:nz], grad_map=to(o.grad_map),
                grad_sources=gs[sl]), others_zero


def run_form(args, w, geom, precision, fold, inputs, log):
    """One plan of the workload: eager steps with per-stage HIP events, then the captured graph
    replayed for the timed region. Returns the plan, the graph and the timings."""
    import torch
    from paper_2406_08703_amd import CapturedEval, EvalBuffers, PsfPlan, evaluate
    from paper_2406_08703_amd import dlx as C
    dev = inputs["dev"]
    c, pm, s, fl, d = inputs["c"], inputs["pm"], inputs["s"], inputs["fl"], inputs["d"]
    t0 = time.perf_counter()
    plan = PsfPlan(geom, dev(w.transmission), dev(w.zbasis), dev(w.map_basis), dev(w.intrapixel),
                   precision=precision, dense_mft=not fold)
    log(f"{precision}: plan created in {time.perf_counter() - t0:.1f} s ({'folded' if fold else 'dense'} MFT, "
        f"workspace {plan.workspace_bytes / 2**30:.2f} GiB, tiles {plan.tiles})")
    ebuf = EvalBuffers(plan)

    def step():   # dlx_eval: forward, loss and adjoint fused per frame chunk
        evaluate(plan, c, pm, s, fl, d, "poisson", w.prior_mu, w.prior_sigma, out=ebuf)

    for i in range(args.warmup):
        step()
        log(f"{precision}: warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    assert plan.sync() == 0
    C.dlx_plan_profile(plan.plan, True)      # eager region, every stage bracketed by HIP events
    t_eager = timed_steps(torch, step, args.steps)[0]
    stages = C.dlx_plan_stage_times(plan.plan)
    C.dlx_plan_profile(plan.plan, False)
    log(f"{precision}: eager {args.steps} steps in {t_eager:.4f} s")
    del ebuf
    t_graph, per_step, cap = None, None, None
    if args.mode == "graph":
        cap = CapturedEval(plan, c, pm, s, fl, d, "poisson", w.prior_mu, w.prior_sigma)
        for _ in range(args.warmup):
            cap.replay()
        t_graph, per_step = timed_steps(torch, cap.replay, args.steps)
        assert plan.sync() == 0
        log(f"{precision}: graph {args.steps} replays in {t_graph:.4f} s")
    table = {}
    for name, (tot, la, ps) in stages.items():
        if la:
            table[name] = dict(ms_per_step=tot / args.steps, launches=la, psfs=ps, avg_launch_ms=tot / la)
    for k, v in table.items():
        log(f"  {k:5s} {v['ms_per_step']:9.4f} ms/step  {v['launches']:5d} launches  avg {v['avg_launch_ms']:.4f} ms")
    return dict(plan=plan, cap=cap, t_eager=t_eager, t_graph=t_graph, per_step=per_step, table=table)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: 200 for c1/c2, 10 otherwise)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default: 5 for c1/c2, 2 otherwise)")
    ap.add_argument("--config", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (then no relative errors are reported either)")
    ap.add_argument("--no-bf16x3", action="store_true", help="skip the BF16x3 record of an FP32 run")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain one-plan-per-PSF timing (c1/c2)")
    ap.add_argument("--dense-mft", action="store_true",
                    help="dense complex MFT products instead of the symmetric fold (the whole run)")
    ap.add_argument("--mode", default="graph", choices=["graph", "eager"],
                    help="graph: the step is one replay of the captured evaluation (dlx_graph_launch)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target host time of the oracle sample")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise copy of MIB MiB (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        x = torch.ones(n, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "dispatches": 3}))
        return
    small = args.config in ("c1", "c2")
    if args.steps is None:
        args.steps = 200 if small else 10
    if args.warmup is None:
        args.warmup = 5 if small else 2
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path shards by frame "
              "with one all-reduce of the flat-field gradient, which this benchmark does not run).", file=sys.stderr)
        sys.exit(2)

    if args.config == "c4":
        return bench_batch(args)
    if args.config == "p0":
        return bench_dither(args)

    import numpy as np
    import torch

    from synth import make_workload, standin_image
    from paper_2406_08703_amd import CapturedEval, EvalBuffers, Geometry, PsfPlan, evaluate

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    w = make_workload(args.config)
    P = w.problem
    w = w.with_data(standin_image(w))
    log(f"workload {args.config}: {WORKLOADS[args.config]}; data: Poisson draw of a smooth stand-in image "
        f"(built in {time.perf_counter() - t0:.1f} s)")

    dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    geom = Geometry(P.n_pupil, P.n_focal, P.oversample, tuple(P.wavelengths), tuple(P.weights), P.n_sources,
                    P.n_frames, P.n_zernike, P.n_map, P.diameter, P.focal_pixel)
    fold = not args.dense_mft
    ep = w.eval_params()
    inputs = dict(dev=dev, c=dev(ep["coeffs"]), pm=dev(ep["phase_map"]), s=dev(ep["sources"]), fl=dev(ep["flat"]),
                  d=dev(w.data))
    f0 = frame_index(P)
    d_f0 = inputs["d"][f0].clone()
    main_form = run_form(args, w, geom, args.precision, fold, inputs, log)
    plan, table = main_form["plan"], main_form["table"]
    t1 = main_form["t_graph"] if main_form["t_graph"] is not None else main_form["t_eager"]
    per_step = main_form["per_step"]
    ms_step = t1 * 1e3 / args.steps
    n_psf = P.n_psf
    evals = n_psf * args.steps / t1
    F_mft = P.mft_flops()
    # algorithmic: the dense two-sided MFT count, forward + adjoint; executed: what the products run
    # (the fused evaluation reuses E, so forward + adjoint only; the fold executes a quarter)
    tf_alg = 2 * F_mft * n_psf / (ms_step * 1e-3) / 1e12
    tf_exec = mft_executed_flops(P, fold) * n_psf / (ms_step * 1e-3) / 1e12
    gemm = {k: v for k, v in table.items() if stage_flops(P, k)}
    roofline = gemm_roofline(P, gemm, plan.tiles, args.precision, args.config, fold)
    gemm_ms = sum(v["ms_per_step"] for v in gemm.values())
    all_ms = sum(v["ms_per_step"] for v in table.values())

    # the split-precision form of the same evaluation, for the speedup and its errors
    split = None
    if args.precision == "fp32" and not args.no_bf16x3 and args.mode == "graph":
        inputs_b = dict(inputs, d=inputs["d"].clone())
        inputs_b["d"][f0] = d_f0
        bf = run_form(args, w, geom, "bf16x3", fold, inputs_b, log)
        ms_b = bf["t_graph"] * 1e3 / args.steps
        gemm_b = {k: v for k, v in bf["table"].items() if stage_flops(P, k)}
        split = {"ms_per_step": round(ms_b, 4), "value": round(n_psf * args.steps / bf["t_graph"], 3),
                 "unit": "PSF evals/s", "step_ms": step_stats(bf["per_step"]),
                 "speedup_vs_fp32": round(ms_step / ms_b, 3),
                 "stage_ms_per_step": {k: round(v["ms_per_step"], 5) for k, v in bf["table"].items()},
                 "tiles": {k: f"{v[0]}x{v[1]}" for k, v in bf["plan"].tiles.items()},
                 "roofline": gemm_roofline(P, gemm_b, bf["plan"].tiles, "bf16x3", args.config, fold),
                 "rel_err_vs_fp64": None}

    cpu, parity = None, None
    if not args.no_cpu_baseline:
        # the FP64 oracle on one full frame (frame f0, every star and wavelength) on the host cores,
        # repeated up to the target time when shorter; its result is also the reference for the
        # relative errors of frame f0
        import oracle as O
        from threadpoolctl import threadpool_info
        prob = O.OracleProblem.from_arrays(P.n_pupil, P.n_focal, P.oversample, P.diameter, P.focal_pixel,
                                           P.wavelengths, P.weights, w.transmission, w.zbasis, w.map_basis,
                                           w.intrapixel)
        sl = slice(f0, f0 + 1)
        dt, reps, ref = 0.0, 0, None
        while dt < args.cpu_seconds or reps == 0:
            t = time.perf_counter()
            ref = O.value_and_grad(prob, ep["coeffs"], ep["phase_map"], ep["sources"][sl], ep["flat"],
                                   w.data[sl], "poisson", w.prior_mu, w.prior_sigma)
            dt += time.perf_counter() - t
            reps += 1
        npsf_frame = P.n_sources * P.n_wavelengths
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        cpu = {"value": round(npsf_frame * reps / dt, 4), "unit": "PSF evals/s", "cores": threads, "kind": "oracle",
               "sample": f"FP64 NumPy oracle forward+loss+gradient of one full frame (frame {f0}: "
                         f"{P.n_sources} star(s) x {P.n_wavelengths} wavelengths = {npsf_frame} PSFs)"
                         f"{f', {reps} times' if reps > 1 else ''}, {dt:.2f} s; the whole {n_psf}-PSF step "
                         f"extrapolated linearly by frames",
               "extrapolated_s_per_step": round(dt / reps * P.n_frames, 3), "host_cpus": os.cpu_count()}
        log(f"cpu baseline: {cpu}")
        phi = ep["sources"][f0, :, 2]
        nz = P.n_zernike
        tol = {"fp32": 1e-5, "bf16x3": 1e-4}
        if main_form["cap"] is not None:
            got, zero = frame_result(main_form["cap"], inputs["d"], d_f0, f0, nz)
            parity = block_errors(dict(got, phi=phi), ref, tol[args.precision], args.precision)
            parity.update(frame=f0, other_frames_exactly_zero=zero)
            log(f"parity of frame {f0} vs FP64 oracle ({args.precision}): {parity}")
        if split is not None:
            got, zero = frame_result(bf["cap"], inputs_b["d"], d_f0, f0, nz)
            split["rel_err_vs_fp64"] = dict(block_errors(dict(got, phi=phi), ref, tol["bf16x3"], "bf16x3"),
                                            frame=f0, other_frames_exactly_zero=zero)
            log(f"parity of frame {f0} vs FP64 oracle (bf16x3): {split['rel_err_vs_fp64']}")
    if split is not None:
        bf["cap"] = None
        bf["plan"].close()

    c, pm, s, fl, d = inputs["c"], inputs["pm"], inputs["s"], inputs["fl"], inputs["d"]

    def timed(fn, k):
        return timed_steps(torch, fn, k)[0]

    separate = None
    if small and not args.no_plain:
        # the three-call boundary path (forward, loss_grad, backward), recomputing the focal fields in
        # backward and with them stored by the forward call (DLX_FLAG_STORE_FIELDS); timing only
        separate = {}
        for sf in (False, True):
            q = PsfPlan(geom, dev(w.transmission), dev(w.zbasis), dev(w.map_basis), dev(w.intrapixel),
                        precision=args.precision, store_fields=sf, dense_mft=not fold)

            def calls():
                B_, m_ = q.forward(c, pm, s, fl)
                _, r_, _ = q.loss_grad(m_, B_, d, fl, "poisson", w.prior_mu, w.prior_sigma)
                q.backward(c, pm, s, fl, r_)

            for _ in range(args.warmup):
                calls()
            t_sep = timed(calls, args.steps)
            assert q.sync() == 0
            q.close()
            separate["stored_fields" if sf else "recompute"] = round(t_sep * 1e3 / args.steps, 4)
        log(f"separate calls ms/step: {separate}")

    plain = None
    if small and P.n_sources == 1 and P.n_frames == 1 and P.n_map == 0 and not args.no_plain:
        # the plain form: one FP32 plan per PSF (here per wavelength), evaluated one after another on
        # the stream, eagerly (per-PSF launches, no batching across PSFs, no graph); timing only
        plans1 = [PsfPlan(Geometry(P.n_pupil, P.n_focal, P.oversample, (lam,), (wt,), 1, 1, P.n_zernike, 0,
                                   P.diameter, P.focal_pixel), dev(w.transmission), dev(w.zbasis), None,
                          dev(w.intrapixel), dense_mft=not fold) for lam, wt in zip(P.wavelengths, P.weights)]
        bufs1 = [EvalBuffers(q) for q in plans1]

        def plain_step():
            for q, b in zip(plans1, bufs1):
                evaluate(q, c, None, s, fl, d, "poisson", w.prior_mu, w.prior_sigma, out=b)

        for _ in range(args.warmup):
            plain_step()
        t_plain = timed(plain_step, args.steps)
        for q in plans1:
            assert q.sync() == 0
            q.close()
        plain = {"ms_per_step": round(t_plain * 1e3 / args.steps, 4), "plans": len(plans1),
                 "speedup_of_measured_form": round(t_plain / t1, 3),
                 "form": "one FP32 plan per PSF, dlx_eval plan after plan on one stream, no graph"}
        log(f"plain fp32: {plain}")

    dense = None
    if small and fold and not args.no_plain:
        # the same captured evaluation with dense complex MFT products (what the fold saves); timing only
        q = PsfPlan(geom, dev(w.transmission), dev(w.zbasis), dev(w.map_basis), dev(w.intrapixel),
                    precision=args.precision, dense_mft=True)
        cq = CapturedEval(q, c, pm, s, fl, d, "poisson", w.prior_mu, w.prior_sigma)
        for _ in range(args.warmup):
            cq.replay()
        t_dense = timed(cq.replay if args.mode == "graph" else
                        (lambda: evaluate(q, c, pm, s, fl, d, "poisson", w.prior_mu, w.prior_sigma)), args.steps)
        assert q.sync() == 0
        cq = None
        q.close()
        dense = {"ms_per_step": round(t_dense * 1e3 / args.steps, 4),
                 "speedup_of_fold": round(t_dense / t1, 3),
                 "form": f"same {args.mode} evaluation, dense complex MFT products"}
        log(f"dense MFT: {dense}")

    out = {"metric": METRIC, "value": round(evals, 3), "unit": "PSF evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "bf16x3", "data": "synthetic",
           "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "psf_per_step": n_psf,
                      "n_pupil": P.n_pupil, "n_focal": P.n_focal, "oversample": P.oversample,
                      "wavelengths": P.n_wavelengths, "sources": P.n_sources, "frames": P.n_frames,
                      "zernikes": P.n_zernike, "flat_pixels": P.n_det ** 2, "precision": args.precision},
           "mft": "symmetric fold" if fold else "dense complex products",
           "mft_tflops": {"algorithmic": round(tf_alg, 3), "executed": round(tf_exec, 3),
                          "algorithmic_over_fp32_mfma_peak": round(tf_alg / FP32_MFMA_PEAK_TFLOPS, 4),
                          "frac_fp32_mfma_peak_executed": round(tf_exec / FP32_MFMA_PEAK_TFLOPS, 4)},
           "mode": args.mode, "step_ms": step_stats(per_step) if per_step else None,
           "eager_ms_per_step": round(main_form["t_eager"] * 1e3 / args.steps, 4),
           "tiles": {k: f"{v[0]}x{v[1]}" for k, v in plan.tiles.items()},
           "stage_ms_per_step": {k: round(v["ms_per_step"], 5) for k, v in table.items()},
           "gemm_share_of_step": round(gemm_ms / all_ms, 4) if all_ms else None,
           "hbm_stages": {k: {"bytes_per_step": hbm_bytes(P, k, table),
                              "GB/s": round(hbm_bytes(P, k, table) / (v["ms_per_step"] * 1e-3) / 1e9, 1),
                              "frac_of_8TB/s": round(hbm_bytes(P, k, table) / (v["ms_per_step"] * 1e-3) / 1e9 /
                                                     HBM_PEAK_GBS, 4)}
                          for k, v in table.items() if stage_bytes(P, k)},
           "roofline": roofline, "rel_err_vs_fp64": parity, "cpu_baseline": cpu, "bf16x3": split,
           "plain_fp32": plain, "dense_mft": dense, "separate_calls_ms_per_step": separate}
    main_form["cap"] = None
    plan.close()
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """The batched configuration: 128 uneven problems, two forms of the same evaluation.

    plain:   one plan per problem, dlx_eval problem after problem on one stream, no graph (FP32);
    batched: one multi-problem plan replayed from one HIP graph, in the precision asked for, in two forms:
             "streams", each problem's own launches spread over concurrent streams, and "grouped"
             (DLX_FLAG_GROUPED), one launch per stage over all problems (a device table maps each
             workgroup to its problem and tile). The faster form gives the line's value.
    The roofline is the grouped form's dominant MFT stage, timed with HIP events on its stream.
    """
    import numpy as np
    import torch

    from synth import make_c4_workloads, standin_image
    from paper_2406_08703_amd import BatchPlan, EvalBuffers, Geometry, PsfPlan, evaluate
    from paper_2406_08703_amd import dlx as C

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ws = [w.with_data(standin_image(w)) for w in make_c4_workloads()]
    log(f"workload c4: {WORKLOADS['c4']}; {len(ws)} problems drawn in {time.perf_counter() - t0:.1f} s")
    geoms = [Geometry(w.problem.n_pupil, w.problem.n_focal, w.problem.oversample, tuple(w.problem.wavelengths),
                      tuple(w.problem.weights), w.problem.n_sources, w.problem.n_frames, w.problem.n_zernike,
                      w.problem.n_map, w.problem.diameter, w.problem.focal_pixel) for w in ws]
    n_psf = sum(w.problem.n_psf for w in ws)
    fold = not args.dense_mft
    F_alg = sum(2.0 * w.problem.mft_flops() * w.problem.n_psf for w in ws)
    F_exec = sum(mft_executed_flops(w.problem, fold) * w.problem.n_psf for w in ws)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32))
    dev = lambda a: t(a).cuda()
    eps = [w.eval_params() for w in ws]
    mu, sigma = ws[0].prior_mu, ws[0].prior_sigma

    def timed(fn, k):
        return timed_steps(torch, fn, k)[0]

    # plain FP32: problem after problem on the current stream
    t1 = time.perf_counter()
    plans = [PsfPlan(g, dev(w.transmission), dev(w.zbasis), dense_mft=not fold) for g, w in zip(geoms, ws)]
    log(f"plain: 128 plans created in {time.perf_counter() - t1:.1f} s")
    pin = [(dev(e["coeffs"]), dev(e["sources"]), dev(e["flat"]), dev(w.data)) for e, w in zip(eps, ws)]
    pbuf = [EvalBuffers(p) for p in plans]

    def plain_step():
        for p, (c, s_, fl, d), b in zip(plans, pin, pbuf):
            evaluate(p, c, None, s_, fl, d, "poisson", mu, sigma, out=b)

    for _ in range(args.warmup):
        plain_step()
    torch.cuda.synchronize()
    t_plain = timed(plain_step, args.steps)
    assert all(p.sync() == 0 for p in plans)
    plain_loss = [float(b.loss[0]) for b in pbuf]
    for p in plans:
        p.close()
    del plans, pbuf, pin
    torch.cuda.empty_cache()
    log(f"plain: {args.steps} steps in {t_plain:.4f} s")

    # batched: one multi-problem plan in each form, an eager region with per-stage events, then one graph
    def batched(grouped):
        t1 = time.perf_counter()
        bp = BatchPlan(geoms, [t(w.transmission) for w in ws], [t(w.zbasis) for w in ws], precision=args.precision,
                       dense_mft=not fold, grouped=grouped)
        form = "grouped" if grouped else "streams"
        log(f"batched {args.precision} {form}: plan created in {time.perf_counter() - t1:.1f} s, "
            f"workspace {bp.workspace_bytes / 2**30:.2f} GiB, tiles {C.dlx_plan_tiles(bp.plan)}")
        c = bp.pack("zernike_coeffs", [t(e["coeffs"]) for e in eps])
        s_ = bp.pack("sources", [t(e["sources"]) for e in eps])
        fl = bp.pack("flat", [t(e["flat"]) for e in eps])
        d = bp.pack("images", [t(w.data) for w in ws])
        out = bp.buffers()
        a = bp.eval_args(c, None, s_, fl, d, out, "poisson", mu, sigma)
        for _ in range(args.warmup):
            bp.evaluate(a)
        torch.cuda.synchronize()
        C.dlx_plan_profile(bp.plan, True)
        t_eager = timed(lambda: bp.evaluate(a), args.steps)
        stages = C.dlx_plan_stage_times(bp.plan)
        C.dlx_plan_profile(bp.plan, False)
        bp.capture(a)
        for _ in range(args.warmup):
            bp.replay()
        t_batch, per_step = timed_steps(torch, bp.replay, args.steps)
        assert bp.sync() == 0
        loss = [float(v[0]) for v in bp.unpack("loss", out["loss"].cpu())]
        tiles = C.dlx_plan_tiles(bp.plan)
        bp.close()
        torch.cuda.empty_cache()
        log(f"batched {form}: {args.steps} replays in {t_batch:.4f} s (eager {t_eager:.4f} s)")
        table = {k: dict(ms_per_step=tot / args.steps, launches=la, psfs=ps, avg_launch_ms=tot / la)
                 for k, (tot, la, ps) in stages.items() if la}
        for k, v in table.items():
            log(f"  {k:5s} {v['ms_per_step']:9.4f} ms/step  {v['launches']:6d} launches  avg {v['avg_launch_ms']:.4f} ms")
        return dict(t=t_batch, per_step=per_step, t_eager=t_eager, table=table, loss=loss, tiles=tiles)

    forms = {"streams": batched(False)}
    if fold:
        forms["grouped"] = batched(True)
    best = min(forms, key=lambda k: forms[k]["t"])
    t_batch, per_step = forms[best]["t"], forms[best]["per_step"]
    loss_dev = max(max(abs(x - y) / abs(y) for x, y in zip(f["loss"], plain_loss)) for f in forms.values())

    ms_step = t_batch * 1e3 / args.steps
    evals = n_psf * args.steps / t_batch
    tf_alg = F_alg / (ms_step * 1e-3) / 1e12
    tf_exec = F_exec / (ms_step * 1e-3) / 1e12
    # roofline: the dominant MFT stage of the grouped form, where one launch covers every problem
    rform = "grouped" if "grouped" in forms else "streams"
    table = forms[rform]["table"]
    stage_flops_all = {k: sum(stage_flops(w.problem, k, fold) * w.problem.n_psf for w in ws)
                       for k in ("F1", "F2", "B3", "B4")}
    gemm = {k: v for k, v in table.items() if k in stage_flops_all}
    dom = max(gemm, key=lambda k: gemm[k]["ms_per_step"])
    dv = gemm[dom]
    per_launch = stage_flops_all[dom] * args.steps / dv["launches"]
    achieved = per_launch / (dv["avg_launch_ms"] * 1e-3) / 1e12
    bf = args.precision == "bf16x3"
    kname = (f"fgemm_group_kernel<{dom}> (one launch over all 128 problems)" if rform == "grouped" else
             f"{'fgemm_kernel' if fold else 'cgemm_kernel'}<{dom}> (launches of one problem, averaged over problems)")
    roofline = {"bound": "mfma", "kernel": kname,
                "achieved": round(3.0 * achieved if bf else achieved, 3),
                "peak": BF16_MFMA_PEAK_TFLOPS if bf else FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round((3.0 * achieved / BF16_MFMA_PEAK_TFLOPS) if bf else (achieved / FP32_MFMA_PEAK_TFLOPS), 4),
                "traffic": None, "flops_per_launch": (3.0 if bf else 1.0) * per_launch,
                "avg_launch_ms": round(dv["avg_launch_ms"], 5)}
    if bf:
        roofline["fp32_equivalent_tflops"] = round(achieved, 3)
        roofline["frac_of_fp32_mfma_peak"] = round(achieved / FP32_MFMA_PEAK_TFLOPS, 4)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        from threadpoolctl import threadpool_info
        done, dt, k = 0, 0.0, 0
        while dt < args.cpu_seconds and k < len(ws):
            w, e = ws[k], eps[k]
            P = w.problem
            prob = O.OracleProblem.from_arrays(P.n_pupil, P.n_focal, P.oversample, P.diameter, P.focal_pixel,
                                               P.wavelengths, P.weights, w.transmission, w.zbasis, None, None)
            t1 = time.perf_counter()
            O.value_and_grad(prob, e["coeffs"], None, e["sources"], e["flat"], w.data, "poisson", mu, sigma)
            dt += time.perf_counter() - t1
            done += P.n_psf
            k += 1
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        cpu = {"value": round(done / dt, 4), "unit": "PSF evals/s", "cores": threads, "kind": "oracle",
               "sample": f"FP64 NumPy oracle forward+loss+gradient of the first {k} of 128 problems "
                         f"({done} PSFs, {dt:.2f} s)", "host_cpus": os.cpu_count()}
        log(f"cpu baseline: {cpu}")

    res = {"metric": METRIC, "value": round(evals, 3), "unit": "PSF evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "bf16x3", "data": "synthetic",
           "config": {"workload": f"c4: {WORKLOADS['c4']}", "problems": len(ws), "psf_per_step": n_psf,
                      "precision": args.precision},
           "mft": "symmetric fold" if fold else "dense complex products",
           "mft_tflops": {"algorithmic": round(tf_alg, 3), "executed": round(tf_exec, 3),
                          "algorithmic_over_fp32_mfma_peak": round(tf_alg / FP32_MFMA_PEAK_TFLOPS, 4),
                          "frac_fp32_mfma_peak_executed": round(tf_exec / FP32_MFMA_PEAK_TFLOPS, 4)},
           "mode": "graph", "batched_form": best, "step_ms": step_stats(per_step),
           "batched_forms": {k: {"ms_per_step": round(f["t"] * 1e3 / args.steps, 4),
                                 "eager_ms_per_step": round(f["t_eager"] * 1e3 / args.steps, 4),
                                 "tiles": {s: f"{v[0]}x{v[1]}" for s, v in f["tiles"].items()},
                                 "stage_ms_per_step": {s: round(v["ms_per_step"], 5) for s, v in f["table"].items()},
                                 "launches_per_step": {s: v["launches"] // args.steps for s, v in f["table"].items()}}
                             for k, f in forms.items()},
           "plain_fp32_ms_per_step": round(t_plain * 1e3 / args.steps, 4),
           "speedup_vs_plain_fp32": round(t_plain / t_batch, 3),
           "max_rel_loss_diff_vs_plain": float(f"{loss_dev:.3e}"),
           "roofline": roofline, "rel_err_vs_fp64": None, "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


def bench_dither(args):
    """The paper's own run in integer-dither mode (one 1064-pixel plane per star and wavelength, five
    1024-pixel frames as its windows), and the same five frames through the per-frame path."""
    import numpy as np
    import torch

    from synth import dithered_standin_image, make_dithered_workload
    from paper_2406_08703_amd import CapturedEval, Geometry, PsfPlan
    from paper_2406_08703_amd import dlx as C

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    w = make_dithered_workload()
    w = w.with_data(dithered_standin_image(w))
    P = w.problem
    log(f"workload p0: {WORKLOADS['p0']}; data: Poisson draw of a smooth stand-in image")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    ep = w.eval_params()
    c, fl, d = dev(ep["coeffs"]), dev(ep["flat"]), dev(w.data)
    results = {}
    for mode in ("dither", "per-frame"):
        dith = mode == "dither"
        geom = Geometry(P.n_pupil, P.oversample * w.n_det, P.oversample, tuple(P.wavelengths), tuple(P.weights),
                        P.n_sources, w.n_frames, P.n_zernike, 0, P.diameter, P.focal_pixel,
                        tuple(map(tuple, w.dithers.tolist())) if dith else (), w.margin if dith else 0)
        plan = PsfPlan(geom, dev(w.transmission), dev(w.zbasis), precision=args.precision,
                       dense_mft=args.dense_mft)
        plan.set_phase_screen(dev(w.phase_screen))
        s = dev(ep["sources"] if dith else w.per_frame_sources(ep["sources"]))
        roof, stages = None, None
        if dith:   # eager pass with per-stage HIP events for the roofline of the dominant GEMM
            from paper_2406_08703_amd import EvalBuffers, evaluate
            eb = EvalBuffers(plan)
            evaluate(plan, c, None, s, fl, d, "poisson", w.prior_mu, w.prior_sigma, out=eb)
            C.dlx_plan_profile(plan.plan, True)
            for _ in range(args.steps):
                evaluate(plan, c, None, s, fl, d, "poisson", w.prior_mu, w.prior_sigma, out=eb)
            torch.cuda.synchronize()
            st = C.dlx_plan_stage_times(plan.plan)
            C.dlx_plan_profile(plan.plan, False)
            gemm = {k: dict(ms_per_step=t / args.steps, launches=la, psfs=ps, avg_launch_ms=t / la)
                    for k, (t, la, ps) in st.items() if la and stage_flops(P, k)}
            roof = gemm_roofline(P, gemm, plan.tiles, args.precision, "p0", not args.dense_mft)
            stages = {k: round(t / args.steps, 5) for k, (t, la, ps) in st.items() if la}
            del eb
        cap = CapturedEval(plan, c, None, s, fl, d, "poisson", w.prior_mu, w.prior_sigma)
        for _ in range(args.warmup):
            cap.replay()
        wall, per = timed_steps(torch, cap.replay, args.steps)
        assert plan.sync() == 0
        loss = float(cap.out.loss.cpu()[0])
        psfs = P.n_sources * P.n_wavelengths * (1 if dith else w.n_frames)
        no = P.n_focal if dith else P.oversample * w.n_det
        flops = 2.0 * 8.0 * no * P.n_pupil * (P.n_pupil + no) * psfs   # dense two-sided MFT count
        hi_, ho_ = (P.n_pupil + 1) // 2, (no + 1) // 2
        exec_flops = (flops if args.dense_mft else
                      8.0 * (ho_ * P.n_pupil * hi_ + no * ho_ * hi_ + hi_ * no * ho_ + hi_ * P.n_pupil * ho_) * psfs)
        results[mode] = dict(ms=wall * 1e3 / args.steps, per=per, psfs=psfs, flops=flops, exec_flops=exec_flops,
                             loss=loss,
                             tiles=plan.tiles, roofline=roof, stages=stages)
        log(f"{mode}: {args.steps} replays in {wall:.4f} s ({psfs} PSFs of {no}x{no} per step)")
        cap = None
        plan.close()
        torch.cuda.empty_cache()
    r = results["dither"]
    ms = r["ms"]
    loss_rel = abs(r["loss"] - results["per-frame"]["loss"]) / abs(results["per-frame"]["loss"])

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        from threadpoolctl import threadpool_info
        big = O.OracleProblem.from_arrays(P.n_pupil, P.n_focal, P.oversample, P.diameter, P.focal_pixel,
                                          P.wavelengths[:1], np.ones(1), w.transmission, w.zbasis,
                                          phase_screen=w.phase_screen)
        ns, dt = 1, 0.0
        while True:
            t1 = time.perf_counter()
            O.value_and_grad_dithered(big, ep["coeffs"], None, ep["sources"][:ns], ep["flat"], w.data, w.dithers,
                                      w.margin, "poisson", w.prior_mu, w.prior_sigma)
            dt = time.perf_counter() - t1
            if dt >= args.cpu_seconds or ns >= P.n_sources:
                break
            ns = min(P.n_sources, max(ns + 1, int(ns * args.cpu_seconds / max(dt, 1e-3) * 0.9)))
        sample = f"the first {ns} of 20 stars at 545 nm"
        npsf, reps = ns, 1
        if ns >= P.n_sources and dt < args.cpu_seconds:
            # every star fits: time the whole run (all wavelengths), repeated up to the target time
            full = O.OracleProblem.from_arrays(P.n_pupil, P.n_focal, P.oversample, P.diameter, P.focal_pixel,
                                               P.wavelengths, P.weights, w.transmission, w.zbasis,
                                               phase_screen=w.phase_screen)
            dt, reps = 0.0, 0
            while dt < args.cpu_seconds:
                t1 = time.perf_counter()
                O.value_and_grad_dithered(full, ep["coeffs"], None, ep["sources"], ep["flat"], w.data, w.dithers,
                                          w.margin, "poisson", w.prior_mu, w.prior_sigma)
                dt += time.perf_counter() - t1
                reps += 1
            npsf = P.n_sources * P.n_wavelengths
            sample = f"the whole run (20 stars, 3 wavelengths), {reps} time(s)"
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        cpu = {"value": round(npsf * reps / dt, 4), "unit": "PSF evals/s", "cores": threads, "kind": "oracle",
               "sample": f"FP64 NumPy oracle, dithered value-and-gradient of {sample} on the 1064-pixel plane, "
                         f"all 5 frames ({npsf * reps} PSFs, {dt:.2f} s)", "host_cpus": os.cpu_count()}
        log(f"cpu baseline: {cpu}")

    out = {"metric": METRIC, "value": round(r["psfs"] / (ms * 1e-3), 3), "unit": "PSF evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "bf16x3",
           "data": "synthetic",
           "config": {"workload": f"p0: {WORKLOADS['p0']}", "psf_per_step": r["psfs"], "frames": w.n_frames,
                      "precision": args.precision},
           "mft": "dense complex products" if args.dense_mft else "symmetric fold",
           "mft_tflops": {"algorithmic": round(r["flops"] / (ms * 1e-3) / 1e12, 3),
                          "executed": round(r["exec_flops"] / (ms * 1e-3) / 1e12, 3),
                          "algorithmic_over_fp32_mfma_peak": round(r["flops"] / (ms * 1e-3) / 1e12 /
                                                                   FP32_MFMA_PEAK_TFLOPS, 4),
                          "frac_fp32_mfma_peak_executed": round(r["exec_flops"] / (ms * 1e-3) / 1e12 /
                                                                FP32_MFMA_PEAK_TFLOPS, 4)},
           "mode": "graph", "step_ms": step_stats(r["per"]), "tiles": {k: f"{v[0]}x{v[1]}" for k, v in r["tiles"].items()},
           "stage_ms_per_step": r["stages"],
           "per_frame_path_ms_per_step": round(results["per-frame"]["ms"], 4),
           "speedup_vs_per_frame_path": round(results["per-frame"]["ms"] / ms, 3),
           "loss_rel_diff_vs_per_frame_path": float(f"{loss_rel:.3e}"),
           "paper_context": {"value_and_grad_s": 2.75, "hardware": "Apple M1 Max CPU, JAX FP32",
                             "source": "Section 4 (optimisation timing)",
                             "ratio": round(2.75 / (ms * 1e-3), 1)},
           "roofline": r["roofline"], "rel_err_vs_fp64": None, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
