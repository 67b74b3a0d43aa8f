"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2406_08703_amd import dlx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "dlx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dlx_[a-z_]+)\s*\(", src)))


def test_header_declares_exactly_the_bound_functions():
    assert header_functions() == sorted(dlx.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    lib = dlx.lib()
    for name in header_functions():
        assert hasattr(lib, name), name


def _desc(**kw):
    base = dict(n_pupil=64, n_focal=64, oversample=2, wavelengths=[600e-9], weights=[1.0], n_sources=1,
                n_frames=1, n_zernike=10, n_map=0, diameter=0.5, focal_pixel=3e-7, dithers=None, margin=0)
    base.update(kw)
    return dlx.make_desc(base["n_pupil"], base["n_focal"], base["oversample"], base["wavelengths"],
                         base["weights"], base["n_sources"], base["n_frames"], base["n_zernike"], base["n_map"],
                         base["diameter"], base["focal_pixel"], base["dithers"], base["margin"])


def test_status_strings():
    for s in range(8):
        assert dlx.dlx_status_string(s).startswith("DLX_")
    assert "unknown" in dlx.dlx_status_string(99)


def test_validate_accepts_a_good_problem():
    d, keep = _desc()
    assert dlx.dlx_validate(d) == dlx.DLX_OK


@pytest.mark.parametrize("kw,code", [
    (dict(n_pupil=1), dlx.DLX_ERR_INVALID_ARG),
    (dict(n_focal=0), dlx.DLX_ERR_INVALID_ARG),
    (dict(oversample=0), dlx.DLX_ERR_INVALID_ARG),
    (dict(n_sources=0), dlx.DLX_ERR_INVALID_ARG),
    (dict(n_frames=0), dlx.DLX_ERR_INVALID_ARG),
    (dict(n_zernike=-1), dlx.DLX_ERR_INVALID_ARG),
    (dict(diameter=0.0), dlx.DLX_ERR_INVALID_ARG),
    (dict(focal_pixel=-1.0), dlx.DLX_ERR_INVALID_ARG),
    (dict(wavelengths=[-5e-7], weights=[1.0]), dlx.DLX_ERR_INVALID_ARG),
    (dict(wavelengths=[float("nan")], weights=[1.0]), dlx.DLX_ERR_INVALID_ARG),
    (dict(n_focal=63, oversample=2), dlx.DLX_ERR_SHAPE),
    (dict(n_pupil=20000), dlx.DLX_ERR_SHAPE),
])
def test_validate_rejects(kw, code):
    d, keep = _desc(**kw)
    assert dlx.dlx_validate(d) == code
    # plan creation fails the same way, synchronously, before any device call
    with pytest.raises(dlx.DlxError) as e:
        dlx.dlx_plan_create(d)
    assert e.value.status == code


def test_validate_null_and_count():
    assert dlx.lib().dlx_validate(None, 1) == dlx.DLX_ERR_INVALID_ARG
    d, keep = _desc()
    assert dlx.dlx_validate(d, 0) == dlx.DLX_ERR_INVALID_ARG


def test_plan_create_rejects_bad_precision_and_flags():
    d, keep = _desc()
    with pytest.raises(dlx.DlxError) as e:
        dlx.dlx_plan_create(d, precision=7)
    assert e.value.status == dlx.DLX_ERR_INVALID_ARG
    with pytest.raises(dlx.DlxError) as e:
        dlx.dlx_plan_create(d, flags=64)   # an undefined bit
    assert e.value.status == dlx.DLX_ERR_INVALID_ARG
    assert (dlx.DLX_FLAG_NO_AUTOTUNE | dlx.DLX_FLAG_SEED_PASS | dlx.DLX_FLAG_STORE_FIELDS
            | dlx.DLX_FLAG_PIXEL_KERNEL | dlx.DLX_FLAG_DENSE_MFT | dlx.DLX_FLAG_GROUPED) == 63


def test_calls_on_null_plan_are_rejected():
    assert dlx.lib().dlx_plan_destroy(None) == dlx.DLX_OK
    assert dlx.dlx_plan_workspace_bytes(0) == 0
    assert dlx.dlx_plan_sync(0) == dlx.DLX_ERR_INVALID_ARG
    with pytest.raises(dlx.DlxError):
        dlx.dlx_psf_forward(0, 1, 1, 0, 1, 0, 1, 1, 0, 1, 1)
    with pytest.raises(dlx.DlxError):
        dlx.dlx_loss_grad(0, 1, 1, 1, 1, 0, 1.0, 0.1, 1, 1, 1)
    with pytest.raises(dlx.DlxError):
        dlx.dlx_psf_backward(0, 1, 1, 0, 1, 0, 1, 1, 0, 1, 1, 0, 1)
    with pytest.raises(dlx.DlxError) as e:
        dlx.dlx_plan_set_phase_screen(0, 0, None)
    assert e.value.status == dlx.DLX_ERR_INVALID_ARG


def test_multi_problem_validation_and_null_plan():
    import ctypes
    good, k1 = _desc()
    bad, k2 = _desc(n_focal=63, oversample=2)
    arr = (dlx.dlx_problem_desc * 3)(good, good, bad)
    assert dlx.lib().dlx_validate(arr, 2) == dlx.DLX_OK
    assert dlx.lib().dlx_validate(arr, 3) == dlx.DLX_ERR_SHAPE
    # one bad problem fails the whole plan, before any device call
    with pytest.raises(dlx.DlxError) as e:
        dlx.dlx_plan_create(arr, 3)
    assert e.value.status == dlx.DLX_ERR_SHAPE
    assert dlx.dlx_plan_problems(0) == 0
    with pytest.raises(dlx.DlxError):
        dlx.dlx_plan_offsets(0, 0)
    assert dlx.lib().dlx_plan_offsets(None, 0, ctypes.byref(dlx.dlx_offsets())) == dlx.DLX_ERR_INVALID_ARG


def test_validate_integer_dither_mode():
    ok, k1 = _desc(n_frames=3, dithers=[(0, 0), (2, -2), (-1, 1)], margin=2)
    assert dlx.dlx_validate(ok) == dlx.DLX_OK
    beyond, k2 = _desc(n_frames=2, dithers=[(0, 0), (3, 0)], margin=2)
    assert dlx.dlx_validate(beyond) == dlx.DLX_ERR_INVALID_ARG
    negative, k3 = _desc(n_frames=1, dithers=[(0, 0)], margin=-1)
    assert dlx.dlx_validate(negative) == dlx.DLX_ERR_INVALID_ARG
    too_big, k4 = _desc(n_frames=1, n_focal=16000, oversample=2, dithers=[(0, 0)], margin=500)
    assert dlx.dlx_validate(too_big) == dlx.DLX_ERR_SHAPE
    with pytest.raises(dlx.DlxError) as e:
        dlx.dlx_plan_create(beyond)
    assert e.value.status == dlx.DLX_ERR_INVALID_ARG


def test_no_alloc_loss_rejects_bad_arguments_before_any_device_work():
    L = dlx.lib()
    nd_big = int(dlx.DLX_NOALLOC_MAX_PIXELS ** 0.5) + 1
    good = (1, 1, 1, 1, dlx.DLX_LOSS_POISSON, 1.0, 0.05, 1, 1, 1, None, None)
    assert L.dlx_loss_grad_noalloc(1, nd_big, *good) == dlx.DLX_ERR_UNSUPPORTED
    assert L.dlx_loss_grad_noalloc(0, 16, *good) == dlx.DLX_ERR_INVALID_ARG
    assert L.dlx_loss_grad_noalloc(1, 0, *good) == dlx.DLX_ERR_INVALID_ARG
    assert L.dlx_loss_grad_noalloc(1, 16, None, *good[1:]) == dlx.DLX_ERR_INVALID_ARG
    assert L.dlx_loss_grad_noalloc(1, 16, 1, 1, 1, 1, 9, 1.0, 0.05, 1, 1, 1, None, None) == dlx.DLX_ERR_INVALID_ARG
    assert L.dlx_loss_grad_noalloc(1, 16, 1, 1, 1, 1, 0, 1.0, 0.0, 1, 1, 1, None, None) == dlx.DLX_ERR_INVALID_ARG


def test_validation_layer_under_address_sanitizer(tmp_path):
    """The host validation layer built on its own with AddressSanitizer and UBSan (g++, host code
    only), driven over good and malformed problem descriptions."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "validate_asan"
    src = os.path.join(ROOT, "paper_2406_08703_amd", "csrc", "validate.cpp")
    drv = os.path.join(ROOT, "tests", "native", "validate_driver.cpp")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), src, drv, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0"))
    assert run.returncode == 0, run.stdout + run.stderr
    assert "validation driver ok" in run.stdout


def test_plan_create_reports_oom_for_a_limit_below_one_frame():
    # the workspace limit is checked against the fixed arrays plus one frame before any device call
    d, keep = _desc(n_pupil=256, n_focal=512, oversample=4, n_frames=4)
    out = ctypes.c_void_p()
    s = dlx.lib().dlx_plan_create(ctypes.byref(d), 1, dlx.DLX_FP32, 0, 1 << 20, ctypes.byref(out))
    assert s == dlx.DLX_ERR_OOM and not out.value


def test_plan_create_reports_oom_when_stored_fields_do_not_fit_the_limit():
    # stored fields need every frame in one chunk: a limit that holds one frame but not four fails
    d, keep = _desc(n_pupil=64, n_focal=64, oversample=2, n_frames=4)
    out = ctypes.c_void_p()
    # fixed arrays 96 KiB and 116 KiB per frame at this size: room for one or two frames, not four
    s = dlx.lib().dlx_plan_create(ctypes.byref(d), 1, dlx.DLX_FP32, dlx.DLX_FLAG_STORE_FIELDS, 300000,
                                  ctypes.byref(out))
    assert s == dlx.DLX_ERR_OOM and not out.value
