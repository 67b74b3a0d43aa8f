"""Torch-facing wrapper of libdlx: device buffers, streams and autograd.

PyTorch supplies device memory and the current HIP stream; every step of
the model, loss and gradient runs in the library's kernels. The wrapper
only checks tensor dtypes/shapes and passes pointers (argument marshalling).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import dlx as _c


@dataclass
class Geometry:
    """Sizes and optics of one problem (the fields of dlx_problem_desc)."""
    n_pupil: int
    n_focal: int
    oversample: int
    wavelengths: tuple
    weights: tuple
    n_sources: int
    n_frames: int
    n_zernike: int
    n_map: int
    diameter: float
    focal_pixel: float
    dithers: tuple = ()      # integer-dither mode: ((dx, dy), ...) per frame, whole detector pixels
    margin: int = 0          # enlarged-plane margin in detector pixels (>= every |dither|)

    @property
    def n_det(self) -> int:
        return self.n_focal // self.oversample

    @property
    def sources_shape(self) -> tuple:
        """[F, S, 3], or [S, 3] in integer-dither mode (one set of stars for all frames)."""
        return (self.n_sources, 3) if self.dithers else (self.n_frames, self.n_sources, 3)


def _f32(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


def _ptr(t):
    return 0 if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class PsfPlan:
    """A libdlx plan plus the static inputs of one problem.

    Static inputs (transmission, Zernike basis, bicubic matrix, intra-pixel
    kernel) are bound once; parameters are passed per call. ``store_fields``
    keeps every PSF's focal field from ``forward`` to the next ``backward``
    (which must get the same parameters), so that pair costs two MFTs per PSF
    instead of three, at the price of holding all PSFs in the workspace.
    ``dense_mft`` computes the MFT as dense complex products instead of the
    symmetric fold (a quarter of the work, same results up to rounding).
    """

    def __init__(self, geom: Geometry, transmission, zbasis, map_basis=None, intrapixel=None,
                 precision: str = "fp32", workspace_limit: int = 0, device="cuda", autotune: bool = True,
                 seed_pass: bool = False, store_fields: bool = False, pixel_kernel: bool = False,
                 dense_mft: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("libdlx needs a ROCm GPU")
        self.geom = geom
        self.device = torch.device(device)
        g = geom
        self.transmission = _f32(transmission, (g.n_pupil, g.n_pupil), "transmission")
        self.zbasis = _f32(zbasis, (g.n_zernike, g.n_pupil, g.n_pupil), "zernike_basis") if g.n_zernike else None
        self.map_basis = _f32(map_basis, (g.n_pupil, g.n_map), "map_basis") if g.n_map else None
        Q = g.oversample
        self.pixel_kernel = pixel_kernel
        self.k_shape = (g.n_det, g.n_det, Q, Q) if pixel_kernel else (Q, Q)
        self.intrapixel = None if intrapixel is None else _f32(intrapixel, self.k_shape, "intrapixel")
        desc, self._keep = _c.make_desc(g.n_pupil, g.n_focal, g.oversample, g.wavelengths, g.weights, g.n_sources,
                                        g.n_frames, g.n_zernike, g.n_map, g.diameter, g.focal_pixel,
                                        g.dithers, g.margin)
        prec = {"fp32": _c.DLX_FP32, "bf16x3": _c.DLX_BF16X3}[precision]
        with torch.cuda.device(self.device):
            flags = ((0 if autotune else _c.DLX_FLAG_NO_AUTOTUNE) | (_c.DLX_FLAG_SEED_PASS if seed_pass else 0)
                     | (_c.DLX_FLAG_STORE_FIELDS if store_fields else 0)
                     | (_c.DLX_FLAG_PIXEL_KERNEL if pixel_kernel else 0)
                     | (_c.DLX_FLAG_DENSE_MFT if dense_mft else 0))
            self.plan = _c.dlx_plan_create(desc, 1, prec, flags, int(workspace_limit))
        self.precision = precision

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "plan", None):
            _c.dlx_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tiles(self) -> dict:
        return _c.dlx_plan_tiles(self.plan)

    @property
    def workspace_bytes(self) -> int:
        return _c.dlx_plan_workspace_bytes(self.plan)

    def sync(self) -> int:
        return _c.dlx_plan_sync(self.plan, _stream(self.device))

    def set_phase_screen(self, screen=None) -> None:
        """Static achromatic pupil phase (radians, [n_pupil, n_pupil]) applied to every later call; None clears."""
        n = self.geom.n_pupil
        t = None if screen is None else _f32(screen, (n, n), "phase_screen")
        _c.dlx_plan_set_phase_screen(self.plan, 0, None if t is None else t.data_ptr(), _stream(self.device))
        self._screen = t  # kept alive until the copy on the stream has run

    # ------------------------------------------------------------------ calls
    def _params(self, coeffs, phase_map, sources, flat):
        g = self.geom
        c = _f32(coeffs, (g.n_zernike,), "zernike_coeffs") if g.n_zernike else None
        pm = _f32(phase_map, (g.n_map, g.n_map), "phase_map") if g.n_map else None
        s = _f32(sources, g.sources_shape, "sources")
        fl = _f32(flat, (g.n_det, g.n_det), "flat")
        return c, pm, s, fl

    def forward(self, coeffs, phase_map, sources, flat, binned=None, model=None):
        """dlx_psf_forward: returns (binned B_f, model m_f), each [F, Nd, Nd] float32."""
        g = self.geom
        c, pm, s, fl = self._params(coeffs, phase_map, sources, flat)
        shp = (g.n_frames, g.n_det, g.n_det)
        binned = torch.empty(shp, dtype=torch.float32, device=self.device) if binned is None else _f32(binned, shp, "binned")
        model = torch.empty(shp, dtype=torch.float32, device=self.device) if model is None else _f32(model, shp, "model")
        _c.dlx_psf_forward(self.plan, _ptr(self.transmission), _ptr(self.zbasis), _ptr(self.map_basis), _ptr(c),
                           _ptr(pm), _ptr(s), _ptr(fl), _ptr(self.intrapixel), _ptr(binned), _ptr(model),
                           _stream(self.device))
        return binned, model

    def loss_grad(self, model, binned, data, flat, kind: str = "poisson", prior_mu: float = 1.0,
                  prior_sigma: float = 0.1, out=None):
        """dlx_loss_grad: returns (loss double[1], r float32 [F,Nd,Nd], grad_flat double [Nd,Nd])."""
        g = self.geom
        shp = (g.n_frames, g.n_det, g.n_det)
        m = _f32(model, shp, "model")
        b = _f32(binned, shp, "binned")
        d = _f32(data, shp, "data")
        fl = _f32(flat, (g.n_det, g.n_det), "flat")
        if out is None:
            loss = torch.empty(1, dtype=torch.float64, device=self.device)
            r = torch.empty(shp, dtype=torch.float32, device=self.device)
            gF = torch.empty((g.n_det, g.n_det), dtype=torch.float64, device=self.device)
        else:
            loss, r, gF = out
        k = {"poisson": _c.DLX_LOSS_POISSON, "chi2": _c.DLX_LOSS_CHI2}[kind]
        _c.dlx_loss_grad(self.plan, _ptr(m), _ptr(b), _ptr(d), _ptr(fl), k, prior_mu, prior_sigma, _ptr(loss),
                         _ptr(r), _ptr(gF), _stream(self.device))
        return loss, r, gF

    def backward(self, coeffs, phase_map, sources, flat, r, out=None, grad_intrapixel=None):
        """dlx_psf_backward: returns (grad_zernike [Nz], grad_map [n_map,n_map] or None, grad_sources [F,S,3]), double.

        ``grad_intrapixel``: an optional float64 device tensor that receives dL/dK ([Q, Q], or
        [Nd, Nd, Q, Q] for a plan with one kernel per pixel)."""
        g = self.geom
        c, pm, s, fl = self._params(coeffs, phase_map, sources, flat)
        rr = _f32(r, (g.n_frames, g.n_det, g.n_det), "dloss_dmodel")
        if out is None:
            gz = torch.empty(max(g.n_zernike, 1), dtype=torch.float64, device=self.device)
            gm = torch.empty((g.n_map, g.n_map), dtype=torch.float64, device=self.device) if g.n_map else None
            gs = torch.empty(g.sources_shape, dtype=torch.float64, device=self.device)
        else:
            gz, gm, gs = out
        gk = None
        if grad_intrapixel is not None:
            if grad_intrapixel.dtype != torch.float64 or tuple(grad_intrapixel.shape) != self.k_shape:
                raise ValueError(f"grad_intrapixel must be a float64 {list(self.k_shape)} tensor")
            gk = grad_intrapixel
        _c.dlx_psf_backward(self.plan, _ptr(self.transmission), _ptr(self.zbasis), _ptr(self.map_basis), _ptr(c),
                            _ptr(pm), _ptr(s), _ptr(fl), _ptr(self.intrapixel), _ptr(rr),
                            _ptr(gz) if g.n_zernike else 0, _ptr(gm), _ptr(gs), _ptr(gk), _stream(self.device))
        return (gz[:g.n_zernike], gm, gs)


class EvalBuffers:
    """Device outputs of one full evaluation (forward, loss, backward)."""

    def __init__(self, plan: "PsfPlan"):
        g, dv = plan.geom, plan.device
        shp = (g.n_frames, g.n_det, g.n_det)
        self.binned = torch.empty(shp, dtype=torch.float32, device=dv)
        self.model = torch.empty(shp, dtype=torch.float32, device=dv)
        self.r = torch.empty(shp, dtype=torch.float32, device=dv)
        self.loss = torch.empty(1, dtype=torch.float64, device=dv)
        self.grad_flat = torch.empty((g.n_det, g.n_det), dtype=torch.float64, device=dv)
        self.grad_zernike = torch.empty(max(g.n_zernike, 1), dtype=torch.float64, device=dv)
        self.grad_map = torch.empty((g.n_map, g.n_map), dtype=torch.float64, device=dv) if g.n_map else None
        self.grad_sources = torch.empty(g.sources_shape, dtype=torch.float64, device=dv)
        self.grad_intrapixel = torch.empty(plan.k_shape, dtype=torch.float64, device=dv)


def _eval_args(plan: "PsfPlan", coeffs, phase_map, sources, flat, data, kind, prior_mu, prior_sigma,
               out: EvalBuffers, intrapixel_grad: bool = False):
    g = plan.geom
    c, pm, s, fl = plan._params(coeffs, phase_map, sources, flat)
    d = _f32(data, (g.n_frames, g.n_det, g.n_det), "data")
    a = _c.dlx_eval_args()
    a.transmission, a.zernike_basis, a.map_basis = _ptr(plan.transmission), _ptr(plan.zbasis), _ptr(plan.map_basis)
    a.zernike_coeffs, a.phase_map, a.sources, a.flat = _ptr(c), _ptr(pm), _ptr(s), _ptr(fl)
    a.intrapixel, a.data = _ptr(plan.intrapixel), _ptr(d)
    a.loss_kind = {"poisson": _c.DLX_LOSS_POISSON, "chi2": _c.DLX_LOSS_CHI2}[kind]
    a.prior_mu, a.prior_sigma = float(prior_mu), float(prior_sigma)
    a.binned, a.model, a.dloss_dmodel, a.loss = _ptr(out.binned), _ptr(out.model), _ptr(out.r), _ptr(out.loss)
    a.grad_flat = _ptr(out.grad_flat)
    a.grad_zernike = _ptr(out.grad_zernike) if g.n_zernike else None
    a.grad_map, a.grad_sources = _ptr(out.grad_map), _ptr(out.grad_sources)
    a.grad_intrapixel = _ptr(out.grad_intrapixel) if intrapixel_grad else None
    keep = (c, pm, s, fl, d)
    return a, keep


def evaluate(plan: "PsfPlan", coeffs, phase_map, sources, flat, data, kind="poisson", prior_mu=1.0, prior_sigma=0.1,
             out: EvalBuffers | None = None, intrapixel_grad: bool = False) -> EvalBuffers:
    """dlx_eval: forward, loss and backward in one call; returns the output buffers
    (``out.grad_intrapixel`` is filled only with ``intrapixel_grad``)."""
    out = out or EvalBuffers(plan)
    a, keep = _eval_args(plan, coeffs, phase_map, sources, flat, data, kind, prior_mu, prior_sigma, out,
                         intrapixel_grad)
    _c.dlx_eval(plan.plan, a, _stream(plan.device))
    return out


class CapturedEval:
    """A full evaluation recorded once into a HIP graph (dlx_graph_capture) and replayed.

    The input tensors are bound at capture time: update them in place
    (``tensor.copy_``) between replays; outputs land in ``self.out``.
    """

    def __init__(self, plan: "PsfPlan", coeffs, phase_map, sources, flat, data, kind="poisson", prior_mu=1.0,
                 prior_sigma=0.1):
        self.plan = plan
        self.out = EvalBuffers(plan)
        self._args, self._keep = _eval_args(plan, coeffs, phase_map, sources, flat, data, kind, prior_mu,
                                            prior_sigma, self.out)
        _c.dlx_graph_capture(plan.plan, self._args)

    def replay(self) -> EvalBuffers:
        _c.dlx_graph_launch(self.plan.plan, _stream(self.plan.device))
        return self.out


class PsfLoss(torch.autograd.Function):
    """L(coeffs, phase_map, sources, flat) with the hand-written adjoint of the whole chain.

    Forward: dlx_psf_forward then dlx_loss_grad (which also yields r and
    dL/dF). Backward: dlx_psf_backward with r; focal fields are recomputed
    in the library, not stored.
    """

    @staticmethod
    def forward(ctx, plan: PsfPlan, data, kind, prior_mu, prior_sigma, coeffs, phase_map, sources, flat):
        B, m = plan.forward(coeffs, phase_map, sources, flat)
        loss, r, gF = plan.loss_grad(m, B, data, flat, kind, prior_mu, prior_sigma)
        ctx.plan = plan
        ctx.has_map = phase_map is not None
        ctx.save_for_backward(coeffs, phase_map if phase_map is not None else torch.empty(0, device=coeffs.device),
                              sources, flat, r, gF)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        coeffs, pm, sources, flat, r, gF = ctx.saved_tensors
        plan = ctx.plan
        gz, gm, gs = plan.backward(coeffs, pm if ctx.has_map else None, sources, flat, r)
        go = grad_out.to(torch.float64)
        to = lambda g, like: None if g is None else (g * go).to(like.dtype)
        return (None, None, None, None, None, to(gz, coeffs), to(gm, pm) if ctx.has_map else None,
                to(gs, sources), to(gF, flat))


def psf_loss(plan: PsfPlan, data, coeffs, phase_map, sources, flat, kind="poisson", prior_mu=1.0, prior_sigma=0.1):
    """Differentiable loss of the forward model (torch autograd entry point)."""
    return PsfLoss.apply(plan, data, kind, prior_mu, prior_sigma, coeffs, phase_map, sources, flat)


class BatchPlan:
    """Many independent problems in one libdlx plan (dlx_plan_create with n_probs > 1).

    Every array crosses the boundary as one flat tensor holding the problems'
    arrays back to back, problem k at the element offsets the plan reports
    (dlx_plan_offsets). ``pack`` builds such a tensor from per-problem
    tensors and ``unpack`` returns per-problem views of one. One call
    evaluates every problem; the library spreads them over concurrent
    streams joined back into the caller's stream, or, with ``grouped``, runs
    each stage as one launch over every problem (DLX_FLAG_GROUPED).
    """

    _FIELDS = ("transmission", "zernike_basis", "map_basis", "zernike_coeffs", "phase_map", "sources", "flat",
               "intrapixel", "images", "loss")

    def __init__(self, geoms, transmissions, zbases, map_bases=None, intrapixels=None, precision: str = "fp32",
                 workspace_limit: int = 0, device="cuda", autotune: bool = True, store_fields: bool = False,
                 dense_mft: bool = False, pixel_kernel: bool = False, grouped: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("libdlx needs a ROCm GPU")
        self.geoms = list(geoms)
        self.pixel_kernel = pixel_kernel
        n = len(self.geoms)
        if n < 1:
            raise ValueError("need at least one problem")
        self.device = torch.device(device)
        descs = (_c.dlx_problem_desc * n)()
        self._keep = []
        for k, g in enumerate(self.geoms):
            d, keep = _c.make_desc(g.n_pupil, g.n_focal, g.oversample, g.wavelengths, g.weights, g.n_sources,
                                   g.n_frames, g.n_zernike, g.n_map, g.diameter, g.focal_pixel,
                                   g.dithers, g.margin)
            descs[k] = d
            self._keep.append(keep)
        prec = {"fp32": _c.DLX_FP32, "bf16x3": _c.DLX_BF16X3}[precision]
        with torch.cuda.device(self.device):
            flags = ((0 if autotune else _c.DLX_FLAG_NO_AUTOTUNE) | (_c.DLX_FLAG_STORE_FIELDS if store_fields else 0)
                     | (_c.DLX_FLAG_DENSE_MFT if dense_mft else 0)
                     | (_c.DLX_FLAG_PIXEL_KERNEL if pixel_kernel else 0)
                     | (_c.DLX_FLAG_GROUPED if grouped else 0))
            self.plan = _c.dlx_plan_create(descs, n, prec, flags, int(workspace_limit))
        self.precision = precision
        self.offsets = [_c.dlx_plan_offsets(self.plan, k) for k in range(_c.dlx_plan_problems(self.plan))]
        self.transmission = self.pack("transmission", transmissions)
        self.zbasis = self.pack("zernike_basis", zbases) if self.total("zernike_basis") else None
        self.map_basis = self.pack("map_basis", map_bases) if self.total("map_basis") else None
        if intrapixels is not None and any(k is None for k in intrapixels):
            raise ValueError("give an intra-pixel kernel for every problem or for none")
        self.intrapixel = None if intrapixels is None else self.pack("intrapixel", intrapixels)

    def shape(self, field: str, k: int) -> tuple:
        g = self.geoms[k]
        return {"transmission": (g.n_pupil, g.n_pupil), "zernike_basis": (g.n_zernike, g.n_pupil, g.n_pupil),
                "map_basis": (g.n_pupil, g.n_map), "zernike_coeffs": (g.n_zernike,),
                "phase_map": (g.n_map, g.n_map), "sources": g.sources_shape,
                "flat": (g.n_det, g.n_det),
                "intrapixel": ((g.n_det, g.n_det, g.oversample, g.oversample) if self.pixel_kernel
                               else (g.oversample, g.oversample)),
                "images": (g.n_frames, g.n_det, g.n_det), "loss": (1,)}[field]

    def total(self, field: str) -> int:
        k = len(self.geoms) - 1
        n = 1
        for s in self.shape(field, k):
            n *= s
        return self.offsets[k][field] + n

    def pack(self, field: str, tensors, dtype=torch.float32) -> torch.Tensor:
        """One flat device tensor holding tensors[k] at problem k's offset."""
        out = torch.zeros(self.total(field), dtype=dtype, device=self.device)
        for k, t in enumerate(tensors):
            shp = self.shape(field, k)
            n = 1
            for s in shp:
                n *= s
            if n == 0:
                continue
            t = torch.as_tensor(t)
            if tuple(t.shape) != shp:
                raise ValueError(f"{field}[{k}] has shape {tuple(t.shape)}, expected {shp}")
            o = self.offsets[k][field]
            out[o:o + n] = t.reshape(-1).to(device=self.device, dtype=dtype)
        return out

    def unpack(self, field: str, flat: torch.Tensor) -> list:
        """Per-problem views of a packed tensor."""
        out = []
        for k in range(len(self.geoms)):
            shp = self.shape(field, k)
            n = 1
            for s in shp:
                n *= s
            o = self.offsets[k][field]
            out.append(flat[o:o + n].view(shp))
        return out

    def buffers(self, intrapixel_grad: bool = False) -> dict:
        """Packed device outputs of one evaluation (with ``intrapixel_grad`` also dL/dK, FP64, packed
        like the intra-pixel kernels)."""
        dv, f32, f64 = self.device, torch.float32, torch.float64
        e = lambda field, dt: torch.empty(max(self.total(field), 1), dtype=dt, device=dv)
        if intrapixel_grad and self.intrapixel is None:
            raise ValueError("dL/dK needs the intra-pixel kernels")
        return dict(binned=e("images", f32), model=e("images", f32), r=e("images", f32), loss=e("loss", f64),
                    grad_flat=e("flat", f64), grad_zernike=e("zernike_coeffs", f64),
                    grad_map=e("phase_map", f64) if self.map_basis is not None else None,
                    grad_sources=e("sources", f64),
                    grad_intrapixel=e("intrapixel", f64) if intrapixel_grad else None)

    def eval_args(self, coeffs, phase_map, sources, flat, data, out: dict, kind="poisson", prior_mu=1.0,
                  prior_sigma=0.1) -> _c.dlx_eval_args:
        """dlx_eval_args over packed parameter tensors (see ``pack``)."""
        for name, t, field in (("coeffs", coeffs, "zernike_coeffs"), ("sources", sources, "sources"),
                               ("flat", flat, "flat"), ("data", data, "images"), ("phase_map", phase_map,
                                                                                  "phase_map")):
            if t is None:
                continue
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() < self.total(field):
                raise ValueError(f"{name} must be a packed contiguous float32 CUDA tensor of {self.total(field)}")
        a = _c.dlx_eval_args()
        a.transmission, a.zernike_basis, a.map_basis = _ptr(self.transmission), _ptr(self.zbasis), _ptr(self.map_basis)
        a.zernike_coeffs, a.phase_map, a.sources, a.flat = _ptr(coeffs), _ptr(phase_map), _ptr(sources), _ptr(flat)
        a.intrapixel, a.data = _ptr(self.intrapixel), _ptr(data)
        a.loss_kind = {"poisson": _c.DLX_LOSS_POISSON, "chi2": _c.DLX_LOSS_CHI2}[kind]
        a.prior_mu, a.prior_sigma = float(prior_mu), float(prior_sigma)
        a.binned, a.model, a.dloss_dmodel, a.loss = _ptr(out["binned"]), _ptr(out["model"]), _ptr(out["r"]), \
            _ptr(out["loss"])
        a.grad_flat, a.grad_zernike = _ptr(out["grad_flat"]), _ptr(out["grad_zernike"])
        a.grad_map, a.grad_sources = _ptr(out["grad_map"]), _ptr(out["grad_sources"])
        a.grad_intrapixel = _ptr(out.get("grad_intrapixel"))
        return a

    def evaluate(self, args: _c.dlx_eval_args) -> None:
        """dlx_eval over every problem, on the current stream."""
        _c.dlx_eval(self.plan, args, _stream(self.device))

    def capture(self, args: _c.dlx_eval_args) -> None:
        """Record dlx_eval over every problem into the plan's HIP graph."""
        _c.dlx_graph_capture(self.plan, args)

    def replay(self) -> None:
        _c.dlx_graph_launch(self.plan, _stream(self.device))

    def sync(self) -> int:
        return _c.dlx_plan_sync(self.plan, _stream(self.device))

    def set_phase_screen(self, problem: int, screen=None) -> None:
        """Static achromatic pupil phase of problem ``problem`` (radians, [n_pupil, n_pupil]); None clears."""
        n = self.geoms[problem].n_pupil
        t = None if screen is None else _f32(screen, (n, n), "phase_screen")
        _c.dlx_plan_set_phase_screen(self.plan, problem, None if t is None else t.data_ptr(), _stream(self.device))
        self._screens = getattr(self, "_screens", {})
        self._screens[problem] = t

    @property
    def workspace_bytes(self) -> int:
        return _c.dlx_plan_workspace_bytes(self.plan)

    def close(self):
        if getattr(self, "plan", None):
            _c.dlx_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
