"""Train the warm-start network on the GPU with the library's own kernels.

Data: seeded pairs of the training family (n ~ U{2000..8000}, Erdos-Renyi or
Chung-Lu with even odds, average degree U{8..20}, edge noise U[0, 0.15], 64-dim
attributes, 5% anchors, eps = 0.02).  For each pair the plain method (fa_align,
cold start, one outer iteration, a long inner solve) gives the row duals b of
the first solve; the target of node i is (b_i - mean(b)) / eps (a constant shift
of b is absorbed by the first a-update, so the gauge is free).  Inputs are the
per-node features of fa_node_features.

Training: mean squared error, Adam, minibatches; forward (fa_mlp_forward),
backward (fa_mlp_backward) and the update (fa_adam_step) all run in the HIP
library; PyTorch only holds the buffers and draws minibatch indices.

Evaluation: on held-out pairs, the first inner solve from the learned start vs
from zero - marginal error after K iterations, the iterations the learned start
needs to reach the cold solve's final error, and the iterations both need to
reach a fixed tolerance (with the argmax agreement of the two plans there).

Two families: "mixed" (the above; the shipped weights/warm_mlp.bin) and "cl",
the benchmark recipe at n = 20,000-40,000 (Chung-Lu, degree 20, d = 128, 2%
anchors; training seeds from 7000, never the benchmark pair's).

Usage: python -m paper_2607_11952_amd.train_warm --pairs 2000 --out <weights>
       python -m paper_2607_11952_amd.train_warm --family cl --pairs 200 --out <weights>
       python -m paper_2607_11952_amd.train_warm --eval-only --weights <weights>
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time

import numpy as np
import torch

from . import api, warm
from .synth import CONFIGS, make_pair

EPS = 0.02


def family(seed: int, n: int = 0):
    r = np.random.default_rng(seed)
    base = CONFIGS["warm_train"]
    return dataclasses.replace(
        base, n1=n or int(r.integers(2000, 8001)), kind="er" if r.random() < 0.5 else "chung_lu",
        avg_deg=float(r.integers(8, 21)), noise=float(r.uniform(0.0, 0.15)), d=64, anchor_frac=0.05, seed=seed,
        eps=EPS)


def family_cl(seed: int, n: int = 0):
    """The benchmark recipe's family at smaller sizes: Chung-Lu, exponent 2.5, average
    degree 20, 10% edge noise, 128-dim attributes with sigma 0.2, 2% anchors, eps 0.02;
    n ~ U{20000..40000} (seeds of their own, never the benchmark pair's)."""
    r = np.random.default_rng(seed)
    return dataclasses.replace(CONFIGS["cl120k"], name="cl_family", n1=n or int(r.integers(20000, 40001)),
                               seed=seed)


FAMILIES = {"mixed": (family, 1000), "cl": (family_cl, 7000)}   # generator, first training seed


def first_solve(inp, inner: int, mlp=None, tol: float = 0.0, fallback: bool = False, probe: int = 0):
    """One outer iteration (the first inner solve); with a network, the learned start
    alone (fallback False) or with the library's cold rerun when it misses tol within
    `probe` iterations (0: the whole budget)."""
    p = api.params(eps=EPS, outer_iters=1, inner_iters=inner, tol=tol, warm_start=mlp is not None,
                   warm_fallback=int(fallback), warm_probe=probe)
    return api.align(inp, p, mlp=mlp)


def pair_data(seed: int, inner: int, device, fam=family):
    pr = make_pair(fam(seed))
    inp = api.AlignInputs.from_pair(pr, device)
    res = first_solve(inp, inner)
    b = res.b.clone()
    t = ((b - b.mean()) / EPS).float()
    inv = api.row_normalize(inp.A1)
    nodes = inp.anchors[:, 0].contiguous()
    F = api.node_features(inp.A1, inv, inp.X1, nodes, None)
    return F, t, float(res.stats.inner_err[0])


def init_params(seed: int, t_mean: float, t_std: float) -> np.ndarray:
    r = np.random.default_rng(seed)
    F, H = 24, 256
    parts = [r.standard_normal((F, H)) * math.sqrt(2.0 / F), np.zeros(H),
             r.standard_normal((H, H)) * math.sqrt(2.0 / H), np.zeros(H),
             r.standard_normal(H) * math.sqrt(1.0 / H), [0.0, t_std, t_mean]]
    p = np.concatenate([np.ravel(x) for x in parts]).astype(np.float32)
    assert p.size == api.mlp_param_count()
    return p


def train(F: torch.Tensor, t: torch.Tensor, epochs: int, batch: int, lr: float, seed: int = 0, log=print):
    dev = F.device
    prm = torch.from_numpy(init_params(seed, float(t.mean()), float(t.std()))).to(dev)
    m = torch.zeros_like(prm)
    v = torch.zeros_like(prm)
    act = api.mlp_act(batch, dev)
    g = torch.Generator(device="cpu").manual_seed(seed)
    N = F.shape[0]
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(dev)
        tot, nb = 0.0, 0
        for s in range(0, N - batch + 1, batch):
            idx = perm[s:s + batch]
            xb, tb = F[idx].contiguous(), t[idx].contiguous()
            api.mlp_forward(prm, xb, act)
            grad, loss = api.mlp_backward(prm, xb, tb, act)
            step += 1
            api.adam_step(prm, grad, m, v, step, lr=lr)
            tot += loss.item() if (nb % 50 == 0) else 0.0
            nb += 1
        y, _ = api.mlp_forward(prm, F[: min(N, 65536)].contiguous())
        mse = float(((y - t[: y.shape[0]]) ** 2).mean())
        hist.append(mse)
        log(f"[train] epoch {ep + 1}/{epochs}: mse {mse:.4f} (target var {float(t.var()):.4f})")
    return prm, hist


def evaluate(prm: torch.Tensor, seeds, n: int, K: int, device, log=print, tol: float = 1e-6, cap: int = 1000,
             probe: int = 0, fam=family):
    rows = []
    for s in seeds:
        pr = make_pair(fam(s, n))
        inp = api.AlignInputs.from_pair(pr, device)
        cold = first_solve(inp, K)
        warm_ = first_solve(inp, K, mlp=prm)
        e_cold, e_warm = float(cold.stats.inner_err[0]), float(warm_.stats.inner_err[0])
        hit = first_solve(inp, K, mlp=prm, tol=e_cold)
        it_warm = int(hit.stats.inner_iters[0])
        agree = float((warm_.argmax == cold.argmax).float().mean())
        # both starts run to the same tolerance (capped)
        ct = first_solve(inp, cap, tol=tol)
        ct_it, ct_err, ct_arg = int(ct.stats.inner_iters[0]), float(ct.stats.inner_err[0]), ct.argmax.clone()
        wt = first_solve(inp, cap, mlp=prm, tol=tol)
        wt_it, wt_err = int(wt.stats.inner_iters[0]), float(wt.stats.inner_err[0])
        agree_tol = float((wt.argmax == ct_arg).float().mean())
        # the product path: learned start, cold rerun when it misses tol (both solves counted)
        fb = first_solve(inp, cap, mlp=prm, tol=tol, fallback=True, probe=probe)
        fb_it, fb_err, fb_fell = int(fb.stats.inner_iters[0]), float(fb.stats.inner_err[0]), int(fb.stats.fell_back)
        agree_fb = float((fb.argmax == ct_arg).float().mean())
        rows.append(dict(seed=s, n=n, K=K, err_cold=e_cold, err_warm=e_warm, iters_warm_to_cold_err=it_warm,
                         argmax_agreement=agree, tol=tol, cap=cap, iters_cold_to_tol=ct_it, err_cold_at_stop=ct_err,
                         iters_warm_to_tol=wt_it, err_warm_at_stop=wt_err, argmax_agreement_at_tol=agree_tol,
                         probe=probe, iters_fallback=fb_it, err_fallback=fb_err, fell_back=fb_fell,
                         argmax_agreement_fallback=agree_fb))
        log(f"[eval] seed {s}: err after {K}: cold {e_cold:.3e} warm {e_warm:.3e}; warm reaches the cold error in "
            f"{it_warm} iterations; argmax agreement {agree:.4f}; to {tol:g}: cold {ct_it} ({ct_err:.2e}) "
            f"warm {wt_it} ({wt_err:.2e}), agreement {agree_tol:.4f}; with fallback {fb_it} ({fb_err:.2e}, "
            f"fell_back {fb_fell})")
    return rows


def summarize(rows):
    f = lambda k: [r[k] for r in rows]
    ic, iw = np.array(f("iters_cold_to_tol"), float), np.array(f("iters_warm_to_tol"), float)
    return dict(pairs=len(rows), mean_err_cold=float(np.mean(f("err_cold"))), mean_err_warm=float(np.mean(f("err_warm"))),
                median_err_ratio=float(np.median(np.array(f("err_cold")) / np.maximum(f("err_warm"), 1e-300))),
                mean_iters_warm_to_cold_err=float(np.mean(f("iters_warm_to_cold_err"))),
                # K cold iterations buy the error the learned start reaches in this many fewer
                speedup_to_cold_err=float(len(rows) * rows[0]["K"] / max(sum(f("iters_warm_to_cold_err")), 1)),
                mean_iters_cold_to_tol=float(ic.mean()), mean_iters_warm_to_tol=float(iw.mean()),
                iteration_ratio=float(ic.sum() / max(iw.sum(), 1.0)),
                min_argmax_agreement_at_tol=float(np.min(f("argmax_agreement_at_tol"))),
                mean_argmax_agreement_at_tol=float(np.mean(f("argmax_agreement_at_tol"))),
                warm_reached_tol=int(sum(r["err_warm_at_stop"] <= r["tol"] for r in rows)),
                cold_reached_tol=int(sum(r["err_cold_at_stop"] <= r["tol"] for r in rows)),
                mean_iters_fallback=float(np.mean(f("iters_fallback"))),
                fallback_reached_tol=int(sum(r["err_fallback"] <= r["tol"] for r in rows)),
                fell_back_pairs=int(sum(r["fell_back"] != 0 for r in rows)),
                iteration_ratio_with_fallback=float(ic.sum() / max(sum(f("iters_fallback")), 1.0)),
                min_argmax_agreement_fallback=float(np.min(f("argmax_agreement_fallback"))))


def markdown(rows, summ, argv: str) -> str:
    """The held-out evaluation as a short markdown record (summary + per-pair table)."""
    r0 = rows[0]
    out = ["# Learned warm start on held-out pairs of its family",
           "",
           f"Command (repository root): `python -m paper_2607_11952_amd.train_warm {argv}`",
           "",
           f"{summ['pairs']} pairs at n = {r0['n']} (seeds {rows[0]['seed']}..{rows[-1]['seed']}, outside the "
           f"training seeds), first inner solve, eps {EPS}; tolerance {r0['tol']:g} with a cap of {r0['cap']} "
           f"iterations; the product path gives the learned start {r0.get('probe', 0) or r0['cap']} iterations, then the "
           f"cold rerun when it has not met the tolerance.",
           "",
           "| | cold start | learned start alone | learned start + cold fallback |",
           "|---|---:|---:|---:|",
           f"| mean iterations (to tol or cap) | {summ['mean_iters_cold_to_tol']:.1f} | {summ['mean_iters_warm_to_tol']:.1f} "
           f"| {summ['mean_iters_fallback']:.1f} |",
           f"| pairs reaching tol | {summ['cold_reached_tol']} | {summ['warm_reached_tol']} | "
           f"{summ['fallback_reached_tol']} |",
           f"| iteration ratio cold / this | 1 | {summ['iteration_ratio']:.2f} | "
           f"{summ['iteration_ratio_with_fallback']:.2f} |",
           f"| min / mean argmax agreement with cold at the stop | - | {summ['min_argmax_agreement_at_tol']:.4f} / "
           f"{summ['mean_argmax_agreement_at_tol']:.4f} | {summ['min_argmax_agreement_fallback']:.4f} |",
           "",
           f"After K = {r0['K']} iterations: mean error cold {summ['mean_err_cold']:.3e}, learned "
           f"{summ['mean_err_warm']:.3e}, median ratio {summ['median_err_ratio']:.1f}; the learned start reaches "
           f"the cold K-iteration error in {summ['mean_iters_warm_to_cold_err']:.1f} iterations on average "
           f"({summ['speedup_to_cold_err']:.2f}x fewer).  Cold rerun used in {summ['fell_back_pairs']} pairs.",
           "",
           "| seed | cold it | cold err | learned it | learned err | +fallback it | +fallback err | kept |",
           "|---:|---:|---:|---:|---:|---:|---:|---|"]
    for r in rows:
        out.append(f"| {r['seed']} | {r['iters_cold_to_tol']} | {r['err_cold_at_stop']:.2e} | {r['iters_warm_to_tol']} "
                   f"| {r['err_warm_at_stop']:.2e} | {r['iters_fallback']} | {r['err_fallback']:.2e} | "
                   f"{'cold' if r['fell_back'] else 'learned'} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--inner", type=int, default=400, help="inner iterations of the target solves")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-pairs", type=int, default=8)
    ap.add_argument("--eval-n", type=int, default=20000)
    ap.add_argument("--eval-k", type=int, default=100)
    ap.add_argument("--eval-seed0", type=int, default=5000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cap", type=int, default=1000)
    ap.add_argument("--probe", type=int, default=50,
                    help="iterations granted to the learned start before the cold rerun (0: the cap)")
    ap.add_argument("--out", default=warm.WEIGHTS)
    ap.add_argument("--family", default="mixed", choices=sorted(FAMILIES),
                    help="mixed: the Erdos-Renyi / Chung-Lu family of n = 2,000-8,000; cl: the benchmark recipe "
                         "(Chung-Lu, degree 20, d = 128, 2% anchors) at n = 20,000-40,000")
    ap.add_argument("--report", default="")
    ap.add_argument("--md", default="", help="markdown record of the evaluation")
    ap.add_argument("--merge", nargs="*", default=None,
                    help="no GPU: merge the eval rows of these report files into one summary (--md / --report)")
    ap.add_argument("--eval-only", action="store_true", help="evaluate --weights, no training")
    ap.add_argument("--weights", default=warm.WEIGHTS)
    args = ap.parse_args()
    if args.merge:
        rows = []
        for f in args.merge:
            with open(f) as fh:
                rows += json.load(fh)["eval"]
        rows.sort(key=lambda r: r["seed"])
        summ = summarize(rows)
        if args.md:
            with open(args.md, "w") as fh:
                fh.write(markdown(rows, summ, " ".join(sys.argv[1:])))
        if args.report:
            with open(args.report, "w") as fh:
                json.dump(dict(eval=rows, summary=summ), fh, indent=1)
        print(json.dumps(summ))
        return
    dev = torch.device("cuda:0")
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.time()
    seeds = range(args.eval_seed0, args.eval_seed0 + args.eval_pairs)
    fam, seed0 = FAMILIES[args.family]
    if args.eval_only:
        prm = torch.from_numpy(warm.read_weights(args.weights)).to(dev)
        rows = evaluate(prm, seeds, args.eval_n, args.eval_k, dev, log=log, tol=args.tol, cap=args.cap,
                        probe=args.probe, fam=fam)
        summ = summarize(rows)
        if args.report:
            with open(args.report, "w") as f:
                json.dump(dict(weights=args.weights, eval=rows, summary=summ, seconds=time.time() - t0), f, indent=1)
        print(json.dumps(summ))
        return
    Fs, ts, errs = [], [], []
    for k in range(args.pairs):
        F, t, e = pair_data(seed0 + k, args.inner, dev, fam)
        Fs.append(F)
        ts.append(t)
        errs.append(e)
        if (k + 1) % 50 == 0:
            log(f"[data] {k + 1}/{args.pairs} pairs, {sum(f.shape[0] for f in Fs)} nodes, "
                f"median target-solve error {np.median(errs):.2e}, {time.time() - t0:.0f}s")
    F = torch.cat(Fs)
    t = torch.cat(ts)
    del Fs, ts
    prm, hist = train(F, t, args.epochs, args.batch, args.lr, log=log)
    warm.save_weights(prm.cpu().numpy(), args.out)
    log(f"[train] saved {args.out}")
    rows = evaluate(prm, seeds, args.eval_n, args.eval_k, dev, log=log, tol=args.tol, cap=args.cap,
                    probe=args.probe, fam=fam)
    summ = summarize(rows)
    rep = dict(pairs=args.pairs, nodes=int(F.shape[0]), target_var=float(t.var()), mse_per_epoch=hist,
               eval=rows, summary=summ, seconds=time.time() - t0)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(dict(final_mse=hist[-1], target_var=float(t.var()), **summ)))


if __name__ == "__main__":
    main()
