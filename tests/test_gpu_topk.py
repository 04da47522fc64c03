"""GPU parity of the plan without a dense buffer: the per-row top-k pass against the
oracle's top-k of the dense plan, and fa_align with the working plan in the C^T
buffer against the same call with a dense plan buffer (results must be identical)."""
import numpy as np
import pytest

from oracle import fastalign_oracle as O
from rank_checks import check_ranks_against_lists
from paper_2607_11952_amd.synth import CONFIGS, PairConfig, make_pair

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api(lib):
    from paper_2607_11952_amd import api as A
    return A


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _inputs(n1, n2, seed):
    r = np.random.default_rng(seed)
    C = (r.random((n1, n2)) * 3).astype(np.float32)
    return C, r.standard_normal(n2) * 0.1, r.standard_normal(n1) * 0.1


@pytest.mark.parametrize("shape,k", [((300, 2500), 1), ((300, 2500), 16), ((257, 3001), 7), ((257, 3001), 64),
                                     ((5, 1030), 33), ((130, 64), 64), ((3, 7), 7)],
                         ids=lambda v: str(v))
def test_plan_topk_vs_oracle(api, shape, k):
    """Indices identical to the oracle's (both order on FP64 exponents; random inputs
    have no ties at that precision), values within FP32 rounding of the oracle's
    plan, and bit for bit the FP32 plan fa_plan writes at the same entries; the
    first column is fa_plan's argmax."""
    n1, n2 = shape
    eps = 0.05
    C, a, b = _inputs(n1, n2, n1 * 7 + n2)
    Cd, ad, bd = _dev(C), _dev(a), _dev(b)
    val, idx = api.plan_topk(Cd, eps, ad, bd, k)
    want_val, want_idx = O.plan_topk(C.astype(np.float64), a, b, eps, k)
    got = idx.cpu().numpy()
    assert np.array_equal(got, want_idx)
    np.testing.assert_allclose(val.cpu().numpy(), want_val, rtol=2e-6, atol=0)
    S, am = api.plan(Cd, eps, ad, bd, argmax=True)
    assert torch.equal(idx[:, 0], am)
    assert torch.equal(val, torch.gather(S, 1, idx.long()))


@pytest.mark.parametrize("n2", [300, 301, 2048])
def test_plan_topk_exact_ties_lowest_column_first(api, n2):
    """Integer costs and zero duals: every row is full of exactly equal exponents, on
    both sides formed from the same FP32 value, so the lists (lowest column first
    among equals, across the workgroup's four partial lists) must match exactly."""
    n1, eps = 67, 0.5
    r = np.random.default_rng(n2)
    C = r.integers(0, 4, size=(n1, n2)).astype(np.float32)
    a, b = np.zeros(n2), np.zeros(n1)
    for k in (5, 37, 64):
        val, idx = api.plan_topk(_dev(C), eps, _dev(a), _dev(b), k)
        want_val, want_idx = O.plan_topk(C.astype(np.float64), a, b, eps, k)
        assert np.array_equal(idx.cpu().numpy(), want_idx), k
        np.testing.assert_allclose(val.cpu().numpy(), want_val, rtol=2e-6)


def _pair_cases():
    return [CONFIGS["er1k"],
            PairConfig("r", 420, "chung_lu", 10.0, noise=0.1, keep_n2=333, d=16, sigma=0.2, anchor_frac=0.08, seed=21)]


@pytest.mark.parametrize("form", ["f32", "bf16"])
@pytest.mark.parametrize("cfg", _pair_cases(), ids=["er1k", "ragged-420x333"])
def test_align_plan_in_ct_is_identical(api, cfg, form):
    """The working plan kept in the C^T buffer (the rebuild writes C only, a transpose
    pass regenerates C^T) gives bit-identical duals, plan, argmax and ranks to the
    run with a dense plan buffer (both keep C^T, so their inner solves run the same
    passes); without any dense plan the top-k lists and ranks agree with that plan."""
    pr = make_pair(cfg)
    truth = pr.truth.astype(np.int32).copy()
    truth[pr.anchors[:, 0]] = -1
    tt = torch.from_numpy(truth).cuda()
    inp = api.AlignInputs.from_pair(pr)
    kw = dict(eps=0.05, outer_iters=4, inner_iters=30, plan_dtype=form, feat_dtype=form, transpose_cost=1)
    ref = api.align(inp, api.params(**kw), truth=tt)
    sh = api.align(inp, api.params(plan_in_ct=1, **kw), truth=tt)
    for f in ("S", "a", "b", "argmax", "rank"):
        assert torch.equal(getattr(ref, f), getattr(sh, f)), f
    assert list(ref.stats.inner_iters)[:4] == list(sh.stats.inner_iters)[:4]
    k = 10
    lean = api.align(inp, api.params(plan_in_ct=1, **kw), truth=tt, topk=k, dense_plan=False)
    assert lean.S is None
    for f in ("a", "b", "argmax", "rank"):
        assert torch.equal(getattr(ref, f), getattr(lean, f)), f
    val, idx = lean.topk_val, lean.topk_idx.long()
    assert torch.equal(idx[:, 0].int(), ref.argmax)
    S = ref.S.float()
    listed = torch.gather(S, 1, idx)
    if form == "f32":
        assert torch.equal(val, listed)
    else:
        assert torch.equal(val.to(torch.bfloat16), ref.S.gather(1, idx))
    rest = S.scatter(1, idx, float("-inf")).max(dim=1).values
    assert torch.all(rest <= listed[:, -1])
    check_ranks_against_lists(ref.rank.cpu().numpy(), truth, val.cpu().numpy(), idx.cpu().numpy())


def test_align_plan_in_ct_argument_checks(api):
    from paper_2607_11952_amd import binding
    pr = make_pair(CONFIGS["er1k"])
    inp = api.AlignInputs.from_pair(pr)
    with pytest.raises(binding.FastAlignError) as ex:
        api.align(inp, api.params(outer_iters=1, inner_iters=1, plan_in_ct=1, transpose_cost=0), dense_plan=False)
    assert ex.value.status == binding.FA_ERR_ARG
    with pytest.raises(binding.FastAlignError) as ex:
        api.align(inp, api.params(outer_iters=1, inner_iters=1, plan_in_ct=1), topk=65, dense_plan=False)
    assert ex.value.status == binding.FA_ERR_ARG
    with pytest.raises(ValueError):
        api.Aligner(inp, api.params(outer_iters=1, inner_iters=1), dense_plan=False)
