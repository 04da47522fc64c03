"""The allocation-free Sinkhorn entry point (static per-GPU scratch) against
fa_sinkhorn with a caller workspace: same kernels, so the same duals, iteration
count and marginal error bit for bit, on two calls in a row (the second smaller,
so the static scratch holds the first call's leftovers), with and without C^T,
and refusal of sizes beyond the static array."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api(lib):
    from paper_2607_11952_amd import api as A
    return A


def _cost(n1, n2, seed):
    r = np.random.default_rng(seed)
    Cm = r.uniform(0.0, 1.0, (n1, n2)) + 0.3 * np.add.outer(r.standard_normal(n1), r.standard_normal(n2))
    return torch.from_numpy(Cm.astype(np.float32)).cuda()


def _noalloc(api, Cm, Ct, eps, a, b, iters, tol):
    from paper_2607_11952_amd import binding
    n1, n2 = Cm.shape
    di = torch.zeros(1, dtype=torch.int32, device="cuda")
    de = torch.zeros(1, dtype=torch.float64, device="cuda")
    binding.load().call("fa_sinkhorn_noalloc", api._ptr(Cm), api._ptr(Ct), n1, n2, float(eps), api._ptr(a),
                        api._ptr(b), int(iters), float(tol), 1, api._ptr(di), api._ptr(de), api._stream())
    torch.cuda.synchronize()
    return int(di.item()), float(de.item())


@pytest.mark.parametrize("transposed", [True, False], ids=["with-Ct", "strips"])
def test_noalloc_sinkhorn_matches_workspace_sinkhorn(api, transposed):
    shapes = [(1500, 1204), (333, 257)] if transposed else [(400, 300), (130, 97)]
    for k, (n1, n2) in enumerate(shapes):      # second call smaller than the first
        Cm = _cost(n1, n2, 7 + k)
        Ct = Cm.t().contiguous() if transposed else None
        eps = 0.05
        for iters, tol in ((40, 0.0), (500, 1e-7)):
            a0 = torch.zeros(n2, dtype=torch.float64, device="cuda")
            b0 = torch.zeros(n1, dtype=torch.float64, device="cuda")
            a1, b1 = a0.clone(), b0.clone()
            it_ws, err_ws = api.sinkhorn(Cm, eps, a0, b0, iters, tol, Ct=Ct)
            it_na, err_na = _noalloc(api, Cm, Ct, eps, a1, b1, iters, tol)
            assert it_na == it_ws and err_na == err_ws, (n1, n2, iters)
            assert torch.equal(a1, a0) and torch.equal(b1, b0), (n1, n2, iters)
            if tol > 0:
                assert err_na <= tol


def test_noalloc_sinkhorn_refuses_sizes_beyond_its_scratch(api):
    from paper_2607_11952_amd import binding
    lib = binding.load()
    n1, n2 = 64, 3_000_000
    need = lib.raw("fa_sinkhorn_noalloc_need")(n1, n2, 1)
    assert need > binding.FA_SINKHORN_NOALLOC_SCRATCH
    assert lib.raw("fa_sinkhorn_noalloc_need")(120000, 120000, 1) <= binding.FA_SINKHORN_NOALLOC_SCRATCH
    Cm = torch.zeros(1, dtype=torch.float32, device="cuda")   # never read: the size check comes first
    a = torch.zeros(1, dtype=torch.float64, device="cuda")
    di = torch.zeros(1, dtype=torch.int32, device="cuda")
    de = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = lib.raw("fa_sinkhorn_noalloc")(api._ptr(Cm), api._ptr(Cm), n1, n2, 0.05, api._ptr(a), api._ptr(a), 10, 0.0,
                                        1, api._ptr(di), api._ptr(de), api._stream())
    assert st == binding.FA_ERR_SHAPE
    assert "static array" in lib.last_error()
