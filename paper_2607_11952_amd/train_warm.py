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
from zero - marginal error after K iterations and the iterations the learned
start needs to reach the cold solve's final error.

Usage: python -m paper_2607_11952_amd.train_warm --pairs 2000 --out <weights>
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
    base = CONFIGS["c4"]
    return dataclasses.replace(
        base, n1=n or int(r.integers(2000, 8001)), kind="er" if r.random() < 0.5 else "chung_lu",
        avg_deg=float(r.integers(8, 21)), noise=float(r.uniform(0.0, 0.15)), d=64, anchor_frac=0.05, seed=seed,
        eps=EPS)


def first_solve(inp, inner: int, mlp=None, tol: float = 0.0):
    p = api.params(eps=EPS, outer_iters=1, inner_iters=inner, tol=tol, warm_start=mlp is not None)
    return api.align(inp, p, mlp=mlp)


def pair_data(seed: int, inner: int, device):
    pr = make_pair(family(seed))
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


def evaluate(prm: torch.Tensor, seeds, n: int, K: int, device, log=print):
    rows = []
    for s in seeds:
        pr = make_pair(family(s, n))
        inp = api.AlignInputs.from_pair(pr, device)
        cold = first_solve(inp, K)
        warm_ = first_solve(inp, K, mlp=prm)
        e_cold, e_warm = float(cold.stats.inner_err[0]), float(warm_.stats.inner_err[0])
        hit = first_solve(inp, K, mlp=prm, tol=e_cold)
        it_warm = int(hit.stats.inner_iters[0])
        agree = float((warm_.argmax == cold.argmax).float().mean())
        rows.append(dict(seed=s, n=n, err_cold=e_cold, err_warm=e_warm, iters_warm_to_cold_err=it_warm,
                         argmax_agreement=agree))
        log(f"[eval] seed {s}: err after {K}: cold {e_cold:.3e} warm {e_warm:.3e}; warm reaches the cold error in "
            f"{it_warm} iterations; argmax agreement {agree:.4f}")
    return rows


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
    ap.add_argument("--out", default=warm.WEIGHTS)
    ap.add_argument("--report", default="")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.time()
    Fs, ts, errs = [], [], []
    for k in range(args.pairs):
        F, t, e = pair_data(1000 + k, args.inner, dev)
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
    rows = evaluate(prm, range(5000, 5000 + args.eval_pairs), args.eval_n, args.eval_k, dev, log=log)
    rep = dict(pairs=args.pairs, nodes=int(F.shape[0]), target_var=float(t.var()), mse_per_epoch=hist,
               eval=rows, seconds=time.time() - t0)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(dict(final_mse=hist[-1], target_var=float(t.var()),
                          mean_err_cold=float(np.mean([r["err_cold"] for r in rows])),
                          mean_err_warm=float(np.mean([r["err_warm"] for r in rows])),
                          mean_iters_warm=float(np.mean([r["iters_warm_to_cold_err"] for r in rows])))))


if __name__ == "__main__":
    main()
