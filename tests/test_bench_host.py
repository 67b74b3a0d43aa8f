"""Host-side arithmetic of the benchmark (no GPU): stage flops, the roofline entry and the
traffic lookup from the committed rocprofv3 summary, including its guard on the GEMM source."""
import hashlib
import os

import pytest

import bench
from synth import make_problem


def test_stage_flops_sum_to_two_mfts_per_psf():
    P = make_problem("c2")
    total = sum(bench.stage_flops(P, k, fold=False) for k in ("F1", "F2", "B3", "B4"))
    assert total == pytest.approx(2.0 * P.mft_flops())
    assert bench.stage_flops(P, "BIN") is None
    # the symmetric fold runs a quarter of the dense products on even sizes
    assert bench.mft_executed_flops(P) == pytest.approx(0.5 * P.mft_flops())
    # odd sizes: halves rounded up (the middle sample has no partner)
    Q = make_problem("c2", n_pupil=5, n_focal=7, oversample=1)
    assert bench.stage_flops(Q, "F1") == 8.0 * 4 * 5 * 3
    assert bench.stage_flops(Q, "B4") == 8.0 * 3 * 5 * 4


def test_roofline_entry_from_launch_times():
    P = make_problem("c2")
    gemm = {"F2": dict(ms_per_step=0.1, launches=10, psfs=200, avg_launch_ms=0.1),
            "B3": dict(ms_per_step=0.2, launches=10, psfs=200, avg_launch_ms=0.2)}
    tiles = {"F1": (64, 32), "F2": (64, 64), "B3": (32, 64), "B4": (64, 32)}
    r = bench.gemm_roofline(P, gemm, tiles, "fp32", "nonexistent-config")
    flops = bench.stage_flops(P, "B3") * 20
    assert r["kernel"] == "fgemm_kernel<3, 1, 2, 0> (B3)"
    assert bench.gemm_roofline(P, gemm, tiles, "fp32", "nonexistent-config", fold=False)["achieved"] == \
        pytest.approx(4 * r["achieved"], rel=1e-3)
    assert r["achieved"] == pytest.approx(flops / 0.2e-3 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3, rel=1e-3)
    assert r["traffic"] is None
    b = bench.gemm_roofline(P, gemm, tiles, "bf16x3", "nonexistent-config")
    assert b["achieved"] == pytest.approx(3 * r["achieved"], rel=1e-3)
    assert b["peak"] == 2500.0


def test_traffic_lookup_matches_the_summary_and_guards_the_source(tmp_path, monkeypatch):
    path = os.path.join(bench.ROOT, "profiles", "traffic_c3_fp32.txt")
    lines = open(path).read().splitlines()
    fields = dict(l.split() for l in lines if l.split()[:1] and l.split()[0] in ("fetch_scale", "write_scale",
                                                                                 "kernel_source_sha256"))
    stage = [l.split() for l in lines if l.startswith("stage B3 ")][0]
    wm, wn = (int(x) for x in stage[2].split("<")[1].rstrip(">").split(",")[1:3])
    want = round(1024 * (float(stage[4]) * float(fields["fetch_scale"]) + float(stage[5]) * float(fields["write_scale"])))
    src = os.path.join(bench.ROOT, "paper_2406_08703_amd", "csrc", "mft_gemm.hip")
    current = hashlib.sha256(open(src, "rb").read()).hexdigest()
    got = bench.measured_traffic("c3", "fp32", "B3", (wm, wn))
    if fields["kernel_source_sha256"] == current:
        assert got == want
    else:
        assert got is None
    # a summary taken from another GEMM source is ignored
    root = tmp_path
    (root / "profiles").mkdir()
    (root / "paper_2406_08703_amd" / "csrc").mkdir(parents=True)
    (root / "paper_2406_08703_amd" / "csrc" / "mft_gemm.hip").write_text("// another kernel\n")
    (root / "profiles" / "traffic_c3_fp32.txt").write_text("\n".join(lines) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic("c3", "fp32", "B3", (wm, wn)) is None
