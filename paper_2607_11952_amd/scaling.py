"""Erdos-Renyi scalability sweep of the whole method on one GPU.

The paper's scalability experiments (§4, scalability analysis) align synthetic
Erdos-Renyi pairs of average degree 10 from 10k to 110k nodes with 20% of the
true pairs as anchors.  This sweep runs the same recipe through fa_align (seeded
stand-ins: G2 a random relabelling with 5% edge noise, 32-dim attributes with
N(0, 0.1^2) noise on G2, eps 0.05, 10 outer x 50 inner iterations) in both
precision forms and records, per size: end-to-end time (HIP events, inputs
resident), inner iterations, final marginal error, Hits@1 / Hits@10 / MRR over
the non-anchor true pairs, and the device memory the call needs (workspace +
plan), from which the largest n that fits in the device's memory follows, with a
dense plan buffer and with the working plan kept in the C^T buffer (no plan buffer).

Usage: python -m paper_2607_11952_amd.scaling [--sizes 10000,20000,...] [--plan-in-ct] [--out sweep.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import api, binding
from .synth import PairConfig, make_pair

SIZES = [10000, 20000, 30000, 40000, 50000, 60000, 70000, 80000, 90000, 100000, 110000]


def recipe(n: int) -> PairConfig:
    return PairConfig(f"er{n // 1000}k", n, "er", 10.0, noise=0.05, d=32, sigma=0.1, anchor_frac=0.2, seed=7,
                      eps=0.05, outer_iters=10, inner_iters=50)


def device_bytes(inp: api.AlignInputs, p) -> int:
    """Workspace plus plan (none when it lives in the C^T buffer) of one fa_align call."""
    n1, n2 = inp.A1.n, inp.A2.n
    plan = 0 if p.plan_in_ct else n1 * n2 * (2 if p.plan_dtype == binding.FA_BF16 else 4)
    return api.workspace_bytes(inp, p) + plan


def largest_n(form: str, capacity: int, plan_in_ct: bool = False, avg_deg: float = 10.0, d: int = 32,
              anchor_frac: float = 0.2) -> int:
    """Largest n (n1 = n2; by default the sweep's recipe) whose fa_align call fits in
    `capacity` bytes (bisection on the library's own workspace query, plus the dense plan
    unless it lives in the C^T buffer; the CSR and attribute inputs add well under 1%
    and are ignored)."""
    lib = api._lib()
    p = api.params(eps=0.05, plan_dtype=form, feat_dtype=form, plan_in_ct=plan_in_ct)
    sb = 0 if plan_in_ct else (2 if form == "bf16" else 4)

    def need(n):
        nnz = int(avg_deg * n)
        return lib.raw("fa_align_workspace_size")(n, n, d, int(anchor_frac * n), nnz, nnz, p) + n * n * sb

    lo, hi = 1000, 2_000_000
    while hi - lo > 100:
        mid = (lo + hi) // 2
        if need(mid) <= capacity:
            lo = mid
        else:
            hi = mid
    return lo


def run(sizes, forms=("bf16", "f32"), log=print, plan_in_ct=False):
    dev = torch.device("cuda:0")
    rows = []
    for n in sizes:
        cfg = recipe(n)
        pr = make_pair(cfg)
        inp = api.AlignInputs.from_pair(pr, dev)
        truth = pr.truth.astype(np.int32).copy()
        truth[pr.anchors[:, 0]] = -1
        tt = torch.from_numpy(truth).to(dev)
        for form in forms:
            p = api.params(eps=cfg.eps, outer_iters=cfg.outer_iters, inner_iters=cfg.inner_iters, plan_dtype=form,
                           feat_dtype=form, plan_in_ct=plan_in_ct)
            al = api.Aligner(inp, p, None, tt, topk=10 if plan_in_ct else 0, dense_plan=not plan_in_ct)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            res = al.run()
            e1.record()
            torch.cuda.synchronize()
            rk = res.rank[res.rank > 0].double()
            row = dict(n=n, form=form, plan_in_ct=bool(plan_in_ct), align_s=e0.elapsed_time(e1) / 1e3, inner_total=int(res.stats.inner_total),
                       marg_err=float(res.stats.marg_err), hits_at_1=float((rk <= 1).double().mean()),
                       hits_at_10=float((rk <= 10).double().mean()), mrr=float((1.0 / rk).mean()),
                       device_gb=device_bytes(inp, p) / 1e9)
            rows.append(row)
            log(f"[sweep] n={n} {form}: {row['align_s']:.3f} s, Hits@1 {row['hits_at_1']:.4f}, "
                f"MRR {row['mrr']:.4f}, {row['device_gb']:.1f} GB")
            del al, res
            torch.cuda.empty_cache()
        del inp
        torch.cuda.empty_cache()
    cap = torch.cuda.get_device_properties(dev).total_memory
    ceiling = {f: largest_n(f, int(cap * 0.97)) for f in forms}
    ceiling.update({f"{f}_plan_in_ct": largest_n(f, int(cap * 0.97), plan_in_ct=True) for f in forms})
    return dict(recipe=dict(kind="er", avg_deg=10, noise=0.05, d=32, sigma=0.1, anchor_frac=0.2, eps=0.05,
                            outer_iters=10, inner_iters=50),
                rows=rows, device_memory_bytes=cap, largest_n_that_fits=ceiling)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default=",".join(map(str, SIZES)))
    ap.add_argument("--forms", default="bf16,f32")
    ap.add_argument("--out", default="")
    ap.add_argument("--md", default="", help="also write a markdown summary of the sweep to this path")
    ap.add_argument("--plan-in-ct", action="store_true",
                    help="keep the working plan in the C^T buffer (no n1 x n2 plan; top-10 lists out)")
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.time()
    out = run([int(x) for x in args.sizes.split(",")], tuple(args.forms.split(",")), log=log,
              plan_in_ct=args.plan_in_ct)
    out["seconds"] = time.time() - t0
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    if args.md:
        with open(args.md, "w") as f:
            f.write(markdown(out, " ".join(sys.argv[1:])))
    print(json.dumps(out))


def markdown(out, argv: str) -> str:
    """Per-size table of a sweep record (time, inner iterations, Hits@1, MRR, device memory)."""
    r = out["recipe"]
    lines = [f"# Erdos-Renyi scalability sweep on one MI355X",
             "",
             f"Command (repository root): `python -m paper_2607_11952_amd.scaling {argv}`",
             "",
             f"Recipe: ER average degree {r['avg_deg']}, {r['noise']:.0%} edge noise, d = {r['d']} "
             f"(sigma {r['sigma']}), {r['anchor_frac']:.0%} anchors, eps {r['eps']}, {r['outer_iters']} outer x "
             f"{r['inner_iters']} inner iterations; times are HIP events around fa_align with inputs resident.",
             "",
             "| n | form | plan in C^T | align s | inner iterations | final L1 error | Hits@1 | Hits@10 | MRR | device GB |",
             "|---:|---|---|---:|---:|---:|---:|---:|---:|---:|"]
    for x in out["rows"]:
        lines.append(f"| {x['n']} | {x['form']} | {'yes' if x['plan_in_ct'] else 'no'} | {x['align_s']:.3f} | "
                     f"{x['inner_total']} | {x['marg_err']:.2e} | {x['hits_at_1']:.4f} | {x['hits_at_10']:.4f} | "
                     f"{x['mrr']:.4f} | {x['device_gb']:.1f} |")
    lines += ["", f"Device memory {out['device_memory_bytes'] / 1e9:.1f} GB; largest n of this recipe that fits "
                  f"(97% of it, the library's workspace query): " +
              ", ".join(f"{k} {v}" for k, v in out["largest_n_that_fits"].items()),
              f"", f"Sweep wall time {out.get('seconds', 0):.0f} s.", ""]
    return "\n".join(lines)


if __name__ == "__main__":
    main()
