"""The autotuner's on-disk cache (DLX_TUNE_CACHE): a plan created with the variable set appends its
tuned tiles (and B4's split and group size) to the file; a later plan of the same shape takes its tiles from the file (here a line
edited by hand to tiles the tuner would not pick), ignores a line whose tiles are not compiled for
their stage, and evaluates the same result whatever the tiles up to the order of partial sums."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _plan(w):
    from tests.gpu_helpers import make_plan
    return make_plan(w)


def test_tune_cache_file_is_written_read_and_validated(tmp_path, monkeypatch):
    from synth import make_workload, standin_image
    from tests.gpu_helpers import run_eval
    from tests.helpers import rel_l2
    print("tune cache", flush=True)
    # a shape no other test uses, so nothing is cached for it yet
    w = make_workload("c2", n_pupil=44, n_focal=52, n_wavelengths=2, noll=tuple(range(2, 7)))
    w = w.with_data(standin_image(w))
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("DLX_TUNE_CACHE", str(path))
    plan = _plan(w)
    tuned = plan.tiles
    ref = run_eval(w, plan=plan)
    plan.close()
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("dlx-tune-v2 ") and " : " in lines[0]
    key, vals = lines[0].split(" : ")
    assert len(vals.split()) == 10
    # a hand-edited line: every stage on the 32 x 32 tile, B4 unsplit, B4 groups of its heuristic size
    path.write_text(f"{key} : 1 1 1 1 1 1 1 1 1 1\n")
    plan = _plan(w)
    assert plan.tiles == {"F1": (32, 32), "F2": (32, 32), "B3": (32, 32), "B4": (32, 32)}
    got = run_eval(w, plan=plan)
    plan.close()
    np.testing.assert_array_equal(got["model"], ref["model"])   # the images do not depend on the tiles
    assert rel_l2(got["grad_coeffs"], ref["grad_coeffs"]) < 1e-6
    # an uncompiled folded FP32 tile (128 x 128) is ignored: the shape is tuned again and appended
    path.write_text(f"{key} : 4 4 1 1 1 1 1 1 1 1\nnot a cache line\n")
    plan = _plan(w)
    assert plan.tiles["F1"] != (128, 128)
    plan.close()
    lines = path.read_text().splitlines()
    assert len(lines) == 3 and lines[2].startswith(key)
    monkeypatch.delenv("DLX_TUNE_CACHE")
    assert "DLX_TUNE_CACHE" not in os.environ
    assert tuned["F1"][0] % 32 == 0
