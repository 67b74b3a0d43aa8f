"""ctypes binding of libdlx (include/dlx.h): same names, argument marshalling only.

Every function here forwards to the HIP library; none computes any part of
the model. The library must have been built (``python -m
paper_2406_08703_amd.build``); loading fails loudly otherwise.

Pointers are passed as integers (device addresses, e.g. ``tensor.data_ptr()``)
and streams as integer ``hipStream_t`` handles (0 = default stream).
"""
from __future__ import annotations

import ctypes
import os

from . import build as _build

DLX_OK = 0
DLX_ERR_INVALID_ARG = 1
DLX_ERR_SHAPE = 2
DLX_ERR_OOM = 3
DLX_ERR_HIP = 4
DLX_ERR_NONFINITE = 5
DLX_ERR_DOMAIN = 6
DLX_ERR_UNSUPPORTED = 7

DLX_FP32 = 0
DLX_BF16X3 = 1
DLX_LOSS_POISSON = 0
DLX_LOSS_CHI2 = 1

DLX_FLAG_NO_AUTOTUNE = 1
DLX_FLAG_SEED_PASS = 2
DLX_FLAG_STORE_FIELDS = 4
DLX_FLAG_PIXEL_KERNEL = 8
DLX_FLAG_DENSE_MFT = 16
DLX_FLAG_GROUPED = 32

# Every symbol include/dlx.h declares.

EXPORTS = ("dlx_validate", "dlx_plan_create", "dlx_plan_destroy", "dlx_plan_workspace_bytes", "dlx_plan_tiles",
           "dlx_plan_sync",
           "dlx_psf_forward", "dlx_loss_grad", "dlx_psf_backward", "dlx_eval", "dlx_graph_capture",
           "dlx_graph_launch", "dlx_plan_profile", "dlx_plan_stage_times", "dlx_status_string",
           "dlx_plan_offsets", "dlx_plan_problems", "dlx_plan_set_phase_screen", "dlx_loss_grad_noalloc")

DLX_NOALLOC_MAX_PIXELS = 4194304

OFFSET_FIELDS = ("transmission", "zernike_basis", "map_basis", "zernike_coeffs", "phase_map", "sources", "flat",
                 "intrapixel", "images", "loss")

STAGES = ("PREP", "F1", "F2", "BIN", "LOSS", "SEED", "B3", "B4", "GRAD")


class dlx_problem_desc(ctypes.Structure):
    _fields_ = [
        ("n_pupil", ctypes.c_int32), ("n_focal", ctypes.c_int32), ("oversample", ctypes.c_int32),
        ("n_wavelengths", ctypes.c_int32), ("n_sources", ctypes.c_int32), ("n_frames", ctypes.c_int32),
        ("n_zernike", ctypes.c_int32), ("n_map", ctypes.c_int32),
        ("diameter_m", ctypes.c_double), ("focal_pixel_rad", ctypes.c_double),
        ("wavelengths_m", ctypes.POINTER(ctypes.c_double)), ("spectral_weights", ctypes.POINTER(ctypes.c_double)),
        ("frame_dithers", ctypes.POINTER(ctypes.c_int32)), ("dither_margin", ctypes.c_int32),
    ]


class dlx_eval_args(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("transmission", "zernike_basis", "map_basis", "zernike_coeffs",
                                                 "phase_map", "sources", "flat", "intrapixel", "data")] + [
        ("loss_kind", ctypes.c_int), ("prior_mu", ctypes.c_double), ("prior_sigma", ctypes.c_double)] + [
        (n, ctypes.c_void_p) for n in ("binned", "model", "dloss_dmodel", "loss", "grad_flat", "grad_zernike",
                                       "grad_map", "grad_sources", "grad_intrapixel")]


class dlx_offsets(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in OFFSET_FIELDS]


class DlxError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {dlx_status_string(status)}")


_LIB = None
_vp = ctypes.c_void_p


def library_path() -> str:
    return _build.LIB


def lib() -> ctypes.CDLL:
    """Load libdlx.so (once). Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"libdlx.so not built at {path}; run `python -m paper_2406_08703_amd.build`")
        L = ctypes.CDLL(path)
        L.dlx_status_string.restype = ctypes.c_char_p
        L.dlx_status_string.argtypes = [ctypes.c_int]
        L.dlx_validate.restype = ctypes.c_int
        L.dlx_validate.argtypes = [ctypes.POINTER(dlx_problem_desc), ctypes.c_int32]
        L.dlx_plan_create.restype = ctypes.c_int
        L.dlx_plan_create.argtypes = [ctypes.POINTER(dlx_problem_desc), ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                                      ctypes.c_size_t, ctypes.POINTER(_vp)]
        L.dlx_plan_destroy.restype = ctypes.c_int
        L.dlx_plan_destroy.argtypes = [_vp]
        L.dlx_plan_workspace_bytes.restype = ctypes.c_size_t
        L.dlx_plan_workspace_bytes.argtypes = [_vp]
        L.dlx_plan_tiles.restype = ctypes.c_int
        L.dlx_plan_tiles.argtypes = [_vp, _vp]
        L.dlx_plan_sync.restype = ctypes.c_int
        L.dlx_plan_sync.argtypes = [_vp, _vp]
        L.dlx_psf_forward.restype = ctypes.c_int
        L.dlx_psf_forward.argtypes = [_vp] * 12
        L.dlx_loss_grad.restype = ctypes.c_int
        L.dlx_loss_grad.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    _vp, _vp, _vp, _vp]
        L.dlx_psf_backward.restype = ctypes.c_int
        L.dlx_psf_backward.argtypes = [_vp] * 15
        L.dlx_eval.restype = ctypes.c_int
        L.dlx_eval.argtypes = [_vp, ctypes.POINTER(dlx_eval_args), _vp]
        L.dlx_graph_capture.restype = ctypes.c_int
        L.dlx_graph_capture.argtypes = [_vp, ctypes.POINTER(dlx_eval_args)]
        L.dlx_graph_launch.restype = ctypes.c_int
        L.dlx_graph_launch.argtypes = [_vp, _vp]
        L.dlx_plan_profile.restype = ctypes.c_int
        L.dlx_plan_profile.argtypes = [_vp, ctypes.c_int32]
        L.dlx_plan_stage_times.restype = ctypes.c_int
        L.dlx_plan_stage_times.argtypes = [_vp, _vp, _vp, _vp]
        L.dlx_plan_offsets.restype = ctypes.c_int
        L.dlx_plan_offsets.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(dlx_offsets)]
        L.dlx_plan_problems.restype = ctypes.c_int32
        L.dlx_plan_problems.argtypes = [_vp]
        L.dlx_plan_set_phase_screen.restype = ctypes.c_int
        L.dlx_plan_set_phase_screen.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
        L.dlx_loss_grad_noalloc.restype = ctypes.c_int
        L.dlx_loss_grad_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
        _LIB = L
    return _LIB


def make_desc(n_pupil, n_focal, oversample, wavelengths, weights, n_sources, n_frames, n_zernike, n_map,
              diameter, focal_pixel, dithers=None, margin=0):
    """Build a dlx_problem_desc; the returned tuple keeps the host arrays alive.

    ``dithers`` [n_frames][2] (dx, dy) whole detector pixels selects the integer-dither mode."""
    nl = len(wavelengths)
    lam = (ctypes.c_double * nl)(*[float(v) for v in wavelengths])
    wts = (ctypes.c_double * len(weights))(*[float(v) for v in weights])
    dith = None
    if dithers is not None and len(dithers):
        flat = [int(v) for pair in dithers for v in pair]
        dith = (ctypes.c_int32 * len(flat))(*flat)
    d = dlx_problem_desc(int(n_pupil), int(n_focal), int(oversample), nl, int(n_sources), int(n_frames),
                         int(n_zernike), int(n_map), float(diameter), float(focal_pixel),
                         ctypes.cast(lam, ctypes.POINTER(ctypes.c_double)),
                         ctypes.cast(wts, ctypes.POINTER(ctypes.c_double)),
                         ctypes.cast(dith, ctypes.POINTER(ctypes.c_int32)) if dith is not None else None,
                         int(margin))
    return d, (lam, wts, dith)


def _chk(status: int, where: str) -> int:
    if status != DLX_OK:
        raise DlxError(status, where)
    return status


def _p(x) -> int | None:
    return None if x is None or x == 0 else int(x)


def dlx_status_string(status: int) -> str:
    return lib().dlx_status_string(int(status)).decode()


def dlx_validate(desc: dlx_problem_desc, n_probs: int = 1) -> int:
    return lib().dlx_validate(ctypes.byref(desc) if desc is not None else None, n_probs)


def dlx_plan_create(desc: dlx_problem_desc, n_probs: int = 1, precision: int = DLX_FP32, flags: int = 0,
                    workspace_limit_bytes: int = 0) -> int:
    """`desc` is one dlx_problem_desc, or a ctypes array of n_probs of them."""
    out = _vp()
    ref = desc if isinstance(desc, ctypes.Array) else ctypes.byref(desc)
    _chk(lib().dlx_plan_create(ref, n_probs, precision, flags, workspace_limit_bytes, ctypes.byref(out)),
         "dlx_plan_create")
    return out.value


def dlx_plan_problems(plan: int) -> int:
    return int(lib().dlx_plan_problems(_p(plan)))


def dlx_plan_offsets(plan: int, problem: int) -> dict:
    """{array: element offset} of problem `problem` inside the packed arrays of a multi-problem plan."""
    o = dlx_offsets()
    _chk(lib().dlx_plan_offsets(_p(plan), int(problem), ctypes.byref(o)), "dlx_plan_offsets")
    return {n: int(getattr(o, n)) for n in OFFSET_FIELDS}


def dlx_plan_destroy(plan: int) -> None:
    _chk(lib().dlx_plan_destroy(_p(plan)), "dlx_plan_destroy")


def dlx_plan_workspace_bytes(plan: int) -> int:
    return int(lib().dlx_plan_workspace_bytes(_p(plan)))


def dlx_plan_tiles(plan: int) -> dict:
    """{stage: (rows, cols)} of each MFT stage's workgroup output tile."""
    t = (ctypes.c_int32 * 8)()
    _chk(lib().dlx_plan_tiles(_p(plan), ctypes.addressof(t)), "dlx_plan_tiles")
    return {k: (32 * t[2 * i], 32 * t[2 * i + 1]) for i, k in enumerate(("F1", "F2", "B3", "B4"))}


def dlx_plan_set_phase_screen(plan: int, problem: int, screen, stream: int = 0) -> None:
    """Copy a static pupil phase screen (device pointer to [Ni][Ni] FP32 radians, or None to clear)."""
    _chk(lib().dlx_plan_set_phase_screen(_p(plan), int(problem), _p(screen), _p(stream)),
         "dlx_plan_set_phase_screen")


def dlx_plan_sync(plan: int, stream: int = 0) -> int:
    """Synchronise and return the device status word (does not raise)."""
    return lib().dlx_plan_sync(_p(plan), _p(stream))


def dlx_psf_forward(plan, transmission, zernike_basis, map_basis, zernike_coeffs, phase_map, sources, flat,
                    intrapixel, binned_out, model_out, stream=0) -> None:
    _chk(lib().dlx_psf_forward(_p(plan), _p(transmission), _p(zernike_basis), _p(map_basis), _p(zernike_coeffs),
                               _p(phase_map), _p(sources), _p(flat), _p(intrapixel), _p(binned_out), _p(model_out),
                               _p(stream)), "dlx_psf_forward")


def dlx_loss_grad(plan, model, binned, data, flat, kind, prior_mu, prior_sigma, loss_out, dloss_dmodel, grad_flat,
                  stream=0) -> None:
    _chk(lib().dlx_loss_grad(_p(plan), _p(model), _p(binned), _p(data), _p(flat), int(kind), float(prior_mu),
                             float(prior_sigma), _p(loss_out), _p(dloss_dmodel), _p(grad_flat), _p(stream)),
         "dlx_loss_grad")


def dlx_loss_grad_noalloc(n_frames, n_det, model, binned, data, flat, kind, prior_mu, prior_sigma, loss_out,
                          dloss_dmodel, grad_flat, status_out=0, stream=0) -> None:
    """dlx_loss_grad without a plan or any device allocation (a fixed library buffer per device)."""
    _chk(lib().dlx_loss_grad_noalloc(int(n_frames), int(n_det), _p(model), _p(binned), _p(data), _p(flat), int(kind),
                                     float(prior_mu), float(prior_sigma), _p(loss_out), _p(dloss_dmodel),
                                     _p(grad_flat), _p(status_out), _p(stream)), "dlx_loss_grad_noalloc")


def dlx_psf_backward(plan, transmission, zernike_basis, map_basis, zernike_coeffs, phase_map, sources, flat,
                     intrapixel, dloss_dmodel, grad_zernike, grad_map, grad_sources, grad_intrapixel=0,
                     stream=0) -> None:
    _chk(lib().dlx_psf_backward(_p(plan), _p(transmission), _p(zernike_basis), _p(map_basis), _p(zernike_coeffs),
                                _p(phase_map), _p(sources), _p(flat), _p(intrapixel), _p(dloss_dmodel),
                                _p(grad_zernike), _p(grad_map), _p(grad_sources), _p(grad_intrapixel), _p(stream)),
         "dlx_psf_backward")


def dlx_plan_profile(plan: int, enable: bool) -> None:
    _chk(lib().dlx_plan_profile(_p(plan), 1 if enable else 0), "dlx_plan_profile")


def dlx_plan_stage_times(plan: int) -> dict:
    """{stage: (total_ms, launches, psfs)} since profiling was enabled or last read."""
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    la = (ctypes.c_int64 * n)()
    ps = (ctypes.c_int64 * n)()
    _chk(lib().dlx_plan_stage_times(_p(plan), ctypes.addressof(ms), ctypes.addressof(la), ctypes.addressof(ps)),
         "dlx_plan_stage_times")
    return {STAGES[i]: (ms[i], la[i], ps[i]) for i in range(n)}


def dlx_eval(plan: int, args: dlx_eval_args, stream: int = 0) -> None:
    _chk(lib().dlx_eval(_p(plan), ctypes.byref(args), _p(stream)), "dlx_eval")


def dlx_graph_capture(plan: int, args: dlx_eval_args) -> None:
    _chk(lib().dlx_graph_capture(_p(plan), ctypes.byref(args)), "dlx_graph_capture")


def dlx_graph_launch(plan: int, stream: int = 0) -> None:
    _chk(lib().dlx_graph_launch(_p(plan), _p(stream)), "dlx_graph_launch")
