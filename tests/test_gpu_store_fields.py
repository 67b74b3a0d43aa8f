"""Stored focal fields (DLX_FLAG_STORE_FIELDS): the backward call after a forward call reuses
the forward's fields instead of recomputing them, and must give the recomputing plan's results
bit for bit; any call in between discards them, and the torch autograd path uses them."""
import numpy as np
import pytest

from tests.test_gpu_parity import workload

pytestmark = pytest.mark.gpu


def _pair(plan, w, r_from=None):
    from tests.gpu_helpers import dev
    p = w.eval_params()
    c, pm, s, fl = dev(p["coeffs"]), dev(p["phase_map"]), dev(p["sources"]), dev(p["flat"])
    B, m = plan.forward(c, pm, s, fl)
    L, r, gF = plan.loss_grad(m, B, dev(w.data), fl, "poisson", w.prior_mu, w.prior_sigma)
    gz, gm, gs = plan.backward(c, pm, s, fl, r if r_from is None else r_from)
    assert plan.sync() == 0
    to = lambda t: None if t is None else t.cpu().numpy()
    return dict(model=to(m), r=to(r), gz=to(gz), gm=to(gm), gs=to(gs)), r


@pytest.mark.parametrize("case", ["c3-small", "c5-small"])
def test_stored_fields_backward_equals_recompute(case):
    from paper_2406_08703_amd import evaluate
    from tests.gpu_helpers import dev, geometry
    from paper_2406_08703_amd import PsfPlan
    print(f"store fields {case}", flush=True)
    w, _ = workload(case)
    mk = lambda sf: PsfPlan(geometry(w), dev(w.transmission), dev(w.zbasis), dev(w.map_basis), dev(w.intrapixel),
                            store_fields=sf)
    ref_plan, plan = mk(False), mk(True)
    ref, r = _pair(ref_plan, w)
    got, _ = _pair(plan, w)
    for k in ("model", "r", "gz", "gm", "gs"):
        if ref[k] is not None:
            assert np.array_equal(got[k], ref[k]), k
    # a second backward without a forward recomputes: same bits
    p = w.eval_params()
    c, pm, s, fl = dev(p["coeffs"]), dev(p["phase_map"]), dev(p["sources"]), dev(p["flat"])
    gz2, _, gs2 = plan.backward(c, pm, s, fl, r)
    assert np.array_equal(gz2.cpu().numpy(), ref["gz"]) and np.array_equal(gs2.cpu().numpy(), ref["gs"])
    # a fused evaluation between forward and backward discards the stored fields
    plan.forward(c, pm, s, fl)
    evaluate(plan, dev(p["coeffs"]), dev(p["phase_map"]), dev(p["sources"]) * 1.01, dev(p["flat"]), dev(w.data))
    gz3, _, gs3 = plan.backward(c, pm, s, fl, r)
    assert plan.sync() == 0
    assert np.array_equal(gz3.cpu().numpy(), ref["gz"]) and np.array_equal(gs3.cpu().numpy(), ref["gs"])
    ref_plan.close()
    plan.close()


def test_stored_fields_in_integer_dither_mode_and_autograd():
    import torch
    from paper_2406_08703_amd import psf_loss
    from tests.gpu_helpers import dev
    from tests.test_gpu_dither import case, plan_for
    print("store fields dither + autograd", flush=True)
    w, _ = case("q1")
    p = w.eval_params()
    outs = []
    for sf in (False, True):
        plan = plan_for(w, store_fields=sf)
        c = dev(p["coeffs"]).requires_grad_()
        s = dev(p["sources"]).requires_grad_()
        fl = dev(p["flat"]).requires_grad_()
        L = psf_loss(plan, dev(w.data), c, None, s, fl, "poisson", w.prior_mu, w.prior_sigma)
        L.backward()
        torch.cuda.synchronize()
        assert plan.sync() == 0
        outs.append([float(L.detach()), c.grad.cpu().numpy(), s.grad.cpu().numpy(), fl.grad.cpu().numpy()])
        plan.close()
    assert outs[0][0] == outs[1][0]
    for a, b in zip(outs[0][1:], outs[1][1:]):
        assert np.array_equal(a, b)
