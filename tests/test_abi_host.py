"""CPU-side checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side CSR builder is bit-exact with the oracle's (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from oracle import fastalign_oracle as O
from paper_2607_11952_amd.synth import CONFIGS, make_pair

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastalign.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fa_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2607_11952_amd import binding
    return binding.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fa_feature_sim", "fa_cost", "fa_sinkhorn", "fa_align"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2607_11952_amd import binding
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib._dll, n)]
    assert not missing, missing
    assert set(names) == set(binding.EXPORTS)


@pytest.mark.parametrize("cfg", ["er1k", "cl20k"])
def test_csr_build_bit_exact_with_oracle(lib, cfg):
    from paper_2607_11952_amd import api
    pr = make_pair(CONFIGS[cfg])
    for n, e in ((pr.n1, pr.edges1), (pr.n2, pr.edges2)):
        rp, ci = api.csr_build(n, e)
        orp, oci = O.build_csr(n, e)
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
        assert rp.dtype == np.int64 and ci.dtype == np.int32


def test_csr_build_edge_cases(lib):
    from paper_2607_11952_amd import api, binding
    # empty graph, isolated nodes, loops and duplicates
    rp, ci = api.csr_build(5, np.zeros((0, 2), np.int64))
    assert list(rp) == [0] * 6 and ci.size == 0
    e = np.array([[0, 0], [1, 2], [2, 1], [1, 2], [4, 1]])
    rp, ci = api.csr_build(5, e)
    orp, oci = O.build_csr(5, e)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    with pytest.raises(binding.FastAlignError) as ex:
        api.csr_build(3, np.array([[0, 3]]))
    assert ex.value.status == binding.FA_ERR_ARG


def test_default_params_and_sizes(lib):
    from paper_2607_11952_amd import api, binding
    p = api.params(eps=0.02)
    assert p.lambda_p == 0.02 and p.eps_anchor == 0.02 and p.check_every == 1
    assert lib.raw("fa_mlp_param_count")() == 24 * 256 + 256 + 256 * 256 + 256 + 256 + 3
    # workspace queries are pure host functions
    assert lib.raw("fa_sinkhorn_workspace_size")(1000, 1000) > 0
    n = lib.raw("fa_align_workspace_size")(1000, 900, 32, 100, 8000, 7000, p)
    assert n > 2 * 1000 * 900 * 4
    # two FP32 intermediates of ceil(rows/64)*64 x n2, whatever the plan's dtype
    want = 2 * 1024 * 900 * 4
    for dt in (binding.FA_F32, binding.FA_BF16):
        assert lib.raw("fa_cost_workspace_size")(1000, 900, dt, 0) == want
    assert lib.raw("fa_cost_workspace_size")(1000, 900, binding.FA_F32, 100) == 2 * 128 * 900 * 4


def test_plan_topk_rejects_bad_arguments_before_any_device_work(lib):
    """k outside [1, min(64, n2)] and null outputs are refused on the host (no GPU)."""
    from paper_2607_11952_amd import binding
    f = lib.raw("fa_plan_topk")
    assert f(None, 4, 8, 0.1, None, None, 0, None, None, None) == binding.FA_ERR_ARG
    assert f(None, 4, 100, 0.1, None, None, 65, None, None, None) == binding.FA_ERR_ARG
    assert f(None, 4, 8, 0.1, None, None, 9, None, None, None) == binding.FA_ERR_ARG
    assert f(None, 4, 8, 0.1, None, None, 3, None, None, None) == binding.FA_ERR_ARG   # null pointers
    assert f(None, 4, 8, -1.0, None, None, 3, None, None, None) == binding.FA_ERR_ARG
    assert f(None, 0, 8, 0.1, None, None, 3, None, None, None) == binding.FA_OK        # no rows: nothing to do


C_CONSUMER = r"""
#include <stdio.h>
#include <string.h>
#include "fastalign.h"

int main(void) {
  fa_params p;
  fa_default_params(&p);
  if (!(p.eps > 0.0) || p.transpose_cost != 0 || p.plan_in_ct != 0 || p.sink_fused != 1) return 2;
  /* triangle 0-1-2 plus a pendant 3-2, a loop and a duplicate */
  const int64_t e[] = {0, 1, 1, 2, 2, 0, 3, 2, 1, 1, 1, 0};
  int64_t rowptr[5], nnz = -1;
  int32_t col[16];
  if (fa_csr_build(4, 6, e, rowptr, col, 16, &nnz) != FA_OK) return 3;
  printf("%lld", (long long)nnz);
  for (int i = 0; i < 5; ++i) printf(" %lld", (long long)rowptr[i]);
  for (int k = 0; k < nnz; ++k) printf(" %d", col[k]);
  printf("\n");
  if (fa_csr_build(4, 1, (const int64_t[]){0, 9}, rowptr, col, 16, &nnz) != FA_ERR_ARG) return 4;
  if (strlen(fa_last_error()) == 0) return 5;
  if (fa_align_workspace_size(100, 80, 8, 5, 600, 500, &p) == 0) return 6;
  if (fa_plan_topk(NULL, 4, 8, 0.1, NULL, NULL, 65, NULL, NULL, NULL) != FA_ERR_ARG) return 7;
  return 0;
}
"""


def test_plain_c_consumer_links_and_runs_host_entry_points(lib, tmp_path):
    """The boundary is a C ABI: a C99 program that includes only include/fastalign.h
    and links libfastalign.so builds with gcc and runs the host-side entry points
    (defaults, the CSR builder against the oracle's CSR, argument rejection with a
    message, the workspace query) on a machine without a GPU."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_2607_11952_amd import binding
    src = tmp_path / "consumer.c"
    src.write_text(C_CONSUMER)
    exe = tmp_path / "consumer"
    libdir = os.path.dirname(binding.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                    "-L", libdir, "-lfastalign", f"-Wl,-rpath,{libdir}"], check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, (out.returncode, out.stderr)
    vals = [int(v) for v in out.stdout.split()]
    e = np.array([[0, 1], [1, 2], [2, 0], [3, 2], [1, 1], [1, 0]])
    rp, ci = O.build_csr(4, e)
    assert vals[0] == rp[-1] and vals[1:6] == list(rp) and vals[6:] == list(ci)


def test_stepwise_and_noalloc_host_checks(lib):
    """Defaults of the new parameters, the static-scratch size query, and argument
    errors of the stepwise entry points, all decided on the host (no GPU)."""
    import ctypes as C
    from paper_2607_11952_amd import api, binding
    p = api.params()
    assert p.dual_start == binding.FA_START_ZERO and p.warm_fallback == 1 and p.warm_probe == 0
    need = lib.raw("fa_sinkhorn_noalloc_need")
    assert 0 < need(120000, 120000, 1) <= binding.FA_SINKHORN_NOALLOC_SCRATCH
    assert need(64, 3_000_000, 1) > binding.FA_SINKHORN_NOALLOC_SCRATCH
    assert need(120000, 120000, 0) > need(120000, 120000, 1)      # column partials without C^T
    assert need(0, 10, 1) == 0
    st = binding.fa_stats()
    # null graphs: refused before any device work
    assert lib.raw("fa_align_step")(None, None, 0, 0, C.byref(p), None, 0, None, None, None, None, None, None,
                                    C.byref(st), None, 0, None) == binding.FA_ERR_ARG
    assert lib.raw("fa_align_end")(None, None, 0, 0, C.byref(p), 0, None, None, None, None, None, None, 0, None,
                                   None, C.byref(st), None, 0, None) == binding.FA_ERR_ARG
