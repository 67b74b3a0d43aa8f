"""dlx_loss_grad_noalloc (no plan, no allocation) against dlx_loss_grad on a plan, through the C ABI.

Both run the same kernels in the same order, so every output must match bit for bit: two calls in
a row, the second with fewer frames and a smaller detector (the fixed buffer keeps the first call's
partials), both loss kinds, and the device status word (set by a clamped model pixel, then clear
again on the next clean call).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def images(F, nd, seed):
    rng = np.random.default_rng(seed)
    binned = rng.uniform(0.5, 50.0, size=(F, nd, nd)).astype(np.float32)
    flat = rng.normal(1.0, 0.05, size=(nd, nd)).astype(np.float32)
    model = (flat[None] * binned).astype(np.float32)
    data = rng.poisson(model).astype(np.float32)
    return model, binned, data, flat


def with_plan(F, nd, model, binned, data, flat, kind):
    """dlx_loss_grad on a plan of F frames of nd x nd pixels (Q = 1, a small pupil)."""
    import torch
    from paper_2406_08703_amd import Geometry, PsfPlan
    g = Geometry(16, nd, 1, (600e-9,), (1.0,), 1, F, 0, 0, 0.5, 6e-7 / nd)
    plan = PsfPlan(g, torch.ones((16, 16), device="cuda"), None, autotune=False)
    t = lambda a: torch.from_numpy(a).cuda()
    L, r, gF = plan.loss_grad(t(model), t(binned), t(data), t(flat), kind, 1.0, 0.05)
    torch.cuda.synchronize()
    status = plan.sync()
    plan.close()
    return float(L.cpu()[0]), r.cpu().numpy(), gF.cpu().numpy(), status


def no_alloc(F, nd, model, binned, data, flat, kind):
    import torch
    from paper_2406_08703_amd import dlx as C
    t = lambda a: torch.from_numpy(a).cuda()
    m, b, d, fl = t(model), t(binned), t(data), t(flat)
    loss = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    r = torch.full((F, nd, nd), -1.0, dtype=torch.float32, device="cuda")
    gF = torch.full((nd, nd), -1.0, dtype=torch.float64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    k = {"poisson": C.DLX_LOSS_POISSON, "chi2": C.DLX_LOSS_CHI2}[kind]
    C.dlx_loss_grad_noalloc(F, nd, m.data_ptr(), b.data_ptr(), d.data_ptr(), fl.data_ptr(), k, 1.0, 0.05,
                            loss.data_ptr(), r.data_ptr(), gF.data_ptr(), status.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return float(loss.cpu()[0]), r.cpu().numpy(), gF.cpu().numpy(), int(status.cpu()[0])


@pytest.mark.parametrize("kind", ["poisson", "chi2"])
def test_no_alloc_loss_grad_equals_plan_loss_grad(kind):
    for F, nd, seed in ((3, 200, 1), (2, 37, 2)):   # the second call smaller than the first
        print(f"no-alloc loss {kind}: {F} frames of {nd} x {nd}", flush=True)
        args = images(F, nd, seed)
        want = with_plan(F, nd, *args, kind)
        got = no_alloc(F, nd, *args, kind)
        assert want[3] == 0 and got[3] == 0
        assert got[0] == want[0]
        assert np.array_equal(got[1], want[1])
        assert np.array_equal(got[2], want[2])


def test_no_alloc_status_word_reports_and_clears():
    from paper_2406_08703_amd import dlx as C
    model, binned, data, flat = images(1, 40, 3)
    model[0, 5, 7] = 0.0
    data[0, 5, 7] = 3.0
    got = no_alloc(1, 40, model, binned, data, flat, "poisson")
    want = with_plan(1, 40, model, binned, data, flat, "poisson")
    assert want[3] == C.DLX_ERR_DOMAIN
    assert got[3] == 2                       # bit 1: model <= 0 under the Poisson loss
    assert got[0] == want[0] and np.array_equal(got[1], want[1])
    clean = images(1, 40, 4)
    assert no_alloc(1, 40, *clean, "poisson")[3] == 0   # the next clean call sees a clear word


def test_no_alloc_rejects_frames_above_its_limit():
    from paper_2406_08703_amd import dlx as C
    nd = int(np.sqrt(C.DLX_NOALLOC_MAX_PIXELS)) + 1
    with pytest.raises(C.DlxError) as e:
        C.dlx_loss_grad_noalloc(1, nd, 1, 1, 1, 1, C.DLX_LOSS_POISSON, 1.0, 0.05, 1, 1, 1, 0, 0)
    assert e.value.status == C.DLX_ERR_UNSUPPORTED
