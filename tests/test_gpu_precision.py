"""The BF16 form against the FP32 form end to end, on the unequal-size precision
pair at full size (Chung-Lu n1 = 60,000 against a 50,000-node induced subgraph of
its noisy copy, d = 128, 5% anchors, eps 0.02, 20 outer x 100 inner iterations,
later solves started from the mean of the earlier duals).

The stated bound: per outer iteration the BF16 form moves each cost entry by at
most lambda_e E 2^-7 + lambda_n 2^-8 (S and the E-set of the SpMM intermediate
rounded to 8 significant bits; sums of non-negative terms), i.e. at most
lambda_n 2^-8 / eps ~ 0.2 nats in the exponent of the plan for the neighbourhood
term at eps = 0.02.  A row whose top plan entry exceeds the second by more than
1 nat in both forms (five times that per-iteration bound) must have the same
argmax in both forms, up to 1% of such rows (the perturbations of successive
outer iterations need not cancel).  Rows below that margin are near-ties - many
are G1 nodes without a partner in the 50,000-node subgraph - and their argmax is
not defined to this precision in either form; they are reported, not judged."""
import numpy as np
import pytest

from paper_2607_11952_amd.synth import CONFIGS, make_pair

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_bf16_form_agrees_with_fp32_on_resolved_rows(lib):
    import gc
    from paper_2607_11952_amd import api, warm
    gc.collect()
    torch.cuda.empty_cache()
    cfg = CONFIGS["cl60k_50k"]
    pr = make_pair(cfg)
    inp = api.AlignInputs.from_pair(pr)
    mlp = warm.load_weights(torch.device("cuda:0"))
    truth = torch.from_numpy(pr.truth).cuda()
    has = truth >= 0
    out = {}
    for form in ("bf16", "f32"):
        bf = form == "bf16"
        p = api.params(eps=cfg.eps, outer_iters=cfg.outer_iters, inner_iters=cfg.inner_iters, tol=1e-6,
                       plan_dtype=form, feat_dtype=form, warm_start=bf and mlp is not None, dual_start="mean")
        res = api.align(inp, p, mlp if bf else None, topk=2)
        v = res.topk_val.double()
        margin = torch.log(v[:, 0] / v[:, 1].clamp_min(1e-300))
        acc = float((res.argmax.long()[has] == truth[has]).float().mean())
        out[form] = (res.argmax.clone(), margin, acc, float(res.stats.marg_err))
        del res
        gc.collect()
        torch.cuda.empty_cache()
    (a_b, m_b, acc_b, e_b), (a_f, m_f, acc_f, e_f) = out["bf16"], out["f32"]
    agree = float((a_b == a_f).float().mean())
    rows = (m_b > 1.0) & (m_f > 1.0)
    frac = float(rows.float().mean())
    agree_res = float((a_b[rows] == a_f[rows]).float().mean())
    agree_matched = float((a_b[has] == a_f[has]).float().mean())
    agree_unmatched = float((a_b[~has] == a_f[~has]).float().mean())
    print(f"[precision] 60k x 50k: argmax agreement {agree:.4f} overall ({agree_matched:.4f} on the "
          f"{int(has.sum())} rows with a partner in G2, {agree_unmatched:.4f} on the {int((~has).sum())} without); "
          f"{frac:.3f} of rows resolved by > 1 nat, agreement there {agree_res:.4f}; accuracy vs truth BF16 "
          f"{acc_b:.4f} FP32 {acc_f:.4f}; final marginal error {e_b:.2e} / {e_f:.2e}")
    assert agree_res >= 0.99
    assert frac >= 0.75
    assert abs(acc_b - acc_f) <= 0.005
    # rows with a partner in G2 mostly resolve; the overall figure mixes in the partnerless
    # near-ties, whose argmax flips with summation order
    assert agree_matched >= 0.97
    del inp
    gc.collect()
    torch.cuda.empty_cache()
