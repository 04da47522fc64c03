"""Benchmark of the FastAlign hot path on one MI355X.

Workload: two Chung-Lu graphs with n1 = n2 = 120,000 (average degree 20, 10% edge
noise), 128-dim attributes, 2% anchors, eps = 0.02, 30 outer iterations, inner
Sinkhorn capped at 100 iterations with the stop rule L1 marginal error <= 1e-6.

A step is one outer iteration of Algorithm 1 on resident state (cost rebuild from
the sparse adjacencies and the dense plan, the inner Sinkhorn solve, the plan),
called through the C ABI (fa_align_step).  The headline form (plan in BF16, FP32
cost and SpMM intermediates, FP64 duals, learned warm start of the first solve
when trained weights are present (50 iterations, then the cold rerun as its
fallback when it has not met the tolerance), later solves
started from the mean of the earlier solves' duals) runs
ONE alignment: fa_align_begin (Phase 1), then outer iterations 0..T-1 as steps
(the first W are the untimed warm-up, the next K are timed together), then
fa_align_end.  `value` is that whole alignment's device time (the metric is an
align time, lower is better); `ms_per_step` the mean of the K timed steps.  The
plain form (FP32 plan, cold starts, the paper's method) is one fa_align call timed
beside it, and an FP32 run with the headline's start policy separates the effect
of precision from that of the starts; then the FP64 oracle on the host cores on a
bounded sample.  Inputs are
resident in HBM before any timed region.  A wall-clock budget skips the optional
legs (plain form, CPU baseline) if they would not fit, and the line is always
printed.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "align time (s) + SpMM HBM GB/s at n=120k: plain FP32 vs BF16+warm start @1e-6"
HBM_PEAK_GBS = 8000.0
KERNELS = ["lse_col_partial", "lse_col_merge", "lse_row", "cost_stage1", "cost_stage2", "plan", "featsim", "lse_col_t",
           "transpose", "topk", "sink_fused"]
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3}   # dense matrix-core peaks of the part
T_START = time.time()


def log(msg):
    print(f"[bench {time.time() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed outer iterations (K)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed outer iterations before them (W)")
    ap.add_argument("--workload", default="cl120k", help="cl120k (default), cl20k or cl60k_50k")
    ap.add_argument("--n", type=int, default=0, help="override n1 (smaller runs of the same recipe)")
    ap.add_argument("--outer", type=int, default=0, help="override the outer iteration count")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cold", action="store_true", help="headline form without the learned warm start")
    ap.add_argument("--weights", default="", help="warm-start network (default: the package's trained network)")
    ap.add_argument("--start", default="mean", choices=["zero", "carry", "mean"],
                    help="headline form: start of the inner solves after the first")
    ap.add_argument("--warm-probe", type=int, default=50,
                    help="iterations granted to the learned start before its cold rerun (0: the whole solve)")
    ap.add_argument("--no-f32-mean", action="store_true",
                    help="skip the FP32 run with the headline's start policy (the precision-only comparison)")
    ap.add_argument("--plan-in-ct", action="store_true",
                    help="keep the working plan in the C^T buffer: no n1 x n2 plan buffer, top-10 lists out")
    ap.add_argument("--budget-s", type=float, default=540.0,
                    help="wall-clock budget: optional legs are skipped when they would not fit")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes for the CPU baseline (0: all)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 4 GiB device-to-device copy first (reference for HBM byte counters)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU run: read two rocprofv3 --pmc csv outputs (FETCH_SIZE, WRITE_SIZE) of "
                         "`bench.py --outer 1 --steps 1 --warmup 0 --no-plain --no-f32-mean --no-cpu "
                         "--calibrate-copy` and write the per-launch HBM bytes of the headline form's kernels "
                         "into profiles/traffic.json (printing a markdown table)")
    return ap.parse_args()


TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


# Kernel class -> the source file that defines it (with the shared headers).
KERNEL_SOURCES = {"lse_col_partial": "fa_sinkhorn.hip", "lse_col_merge": "fa_sinkhorn.hip", "lse_row": "fa_sinkhorn.hip",
                  "lse_col_t": "fa_sinkhorn.hip", "featsim": "fa_gemm.hip",
                  "plan": "fa_sinkhorn.hip", "cost_stage1": "fa_spmm.hip", "cost_stage2": "fa_spmm.hip",
                  "transpose": "fa_topk.hip", "topk": "fa_topk.hip", "sink_fused": "fa_sinkhorn.hip"}


def source_digest(kernel=None):
    """Digest of a kernel's source file and the shared headers (all sources if kernel is None);
    counter readings are valid only for the code they were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2607_11952_amd", "csrc")
    files = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".h")))
    if kernel is not None:
        files = [f for f in files if f.endswith(".h") or f == KERNEL_SOURCES[kernel]]
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter runs, or None if absent or stale."""
    try:
        with open(TRAFFIC) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("workload") != workload or k.get("source_digest") != source_digest(kernel):
        return None
    return k.get("bytes_per_launch")


def algorithmic_bytes(kind, n1, n2, nnz1, nnz2, chunk, sbytes, zpair, transposed=True):
    """Compulsory HBM bytes per launch of each kernel class (see the design notes)."""
    N = n1 * n2
    if kind in ("lse_col_partial", "lse_row", "lse_col_t", "sink_fused"):
        return 4 * N + 8 * (n1 + n2)                 # one FP32 pass over C (or C^T) + both dual vectors
    if kind == "lse_col_merge":
        return 8 * n2 * 3
    if kind == "cost_stage1":
        return sbytes * n1 * n2 + zpair * chunk * n2   # S read once + both Z sets written (one chunk)
    if kind == "cost_stage2":
        # Z read + C_node, C_prev read + C written (+ C^T written for the transposed column pass)
        return zpair * chunk * n2 + 12 * chunk * n2 + (4 * chunk * n2 if transposed else 0)
    if kind == "plan":
        return (4 + sbytes) * N
    if kind == "featsim":
        return 4 * N          # C_node written once (operands are a few hundred MB)
    if kind == "transpose":
        return 8 * N          # C read, C^T written
    if kind == "topk":
        return 4 * N + 8 * (n1 + n2)
    return 0


def n_chunk(n1, n2, zbytes):
    cap = 16.0 * 2**30
    cr = min(n1, int(cap // max(2.0 * n2 * zbytes, 1.0)))
    cr = max(64, cr // 64 * 64)
    return min(cr, n1)


def kernel_table(st, pair, nnz1, nnz2, p, binding):
    """Per kernel class: launches, device time and algorithmic rate from fa_stats' HIP-event timings."""
    sb = 2 if p.plan_dtype == binding.FA_BF16 else 4
    chunk = n_chunk(pair.n1, pair.n2, 4)  # chunk rows are sized for an FP32 intermediate in both forms
    chunk = pair.n1 / math.ceil(pair.n1 / chunk)  # mean rows per stage launch (the last chunk is short)
    out = {}
    for k, name in enumerate(KERNELS):
        calls = int(st.kernel_calls[k])
        if calls == 0:
            continue
        avg_ms = st.kernel_ms[k] / calls
        # bytes of one Z entry over both value sets: FP32 N-set + E-set in the form's plan type
        by = algorithmic_bytes(name, pair.n1, pair.n2, nnz1, nnz2, chunk, sb, 4 + sb, bool(p.transpose_cost))
        out[name] = dict(calls=calls, total_ms=st.kernel_ms[k], avg_ms=avg_ms, algorithmic_bytes=by,
                         gbps=by / (avg_ms * 1e-3) / 1e9)
        if name == "featsim":
            fl = 2.0 * pair.n1 * pair.n2 * (pair.X1.shape[1] + len(pair.anchors))
            fdt = "bf16" if p.feat_dtype == binding.FA_BF16 else "f32"
            out[name].update(flops=fl, tflops=fl / (avg_ms * 1e-3) / 1e12, dtype=fdt,
                             peak_tflops=MFMA_PEAK_TFLOPS[fdt],
                             frac_of_peak=fl / (avg_ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[fdt])
    return out


# kernel class of the headline form -> the kernel's name prefix in a rocprofv3 record
KERNEL_NAMES = {"sink_fused": "fa::k_sink_fused<4, 2>", "lse_col_t": "fa::k_lse_col_t<4, 8>",
                "lse_col_partial": "fa::k_lse_col_partial<4, 4>", "lse_row": "fa::k_lse_row<4, 8>",
                "cost_stage1": "fa::k_stage1<unsigned short, true, 2, 8, true>",
                "cost_stage2": "fa::k_stage2<true, true>", "plan": "fa::k_plan<4, unsigned short>",
                "featsim": "fa::k_featsim_dma"}


def _counter_rows(d):
    """(kernel name, grid size, counter value) per dispatch from a rocprofv3 csv output tree."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    per = {}
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                key = (f, int(r.get("Dispatch_Id") or r.get("Correlation_Id")))
                name = r["Kernel_Name"]
                if name.startswith("void "):
                    name = name[5:]
                ent = per.setdefault(key, [name, int(r.get("Grid_Size", 0) or 0), 0.0])
                ent[2] += float(r["Counter_Value"])
    return [per[k] for k in sorted(per)]   # dispatch order


def ingest_counters(fetch_dir, write_dir, workload="cl120k:120000x120000"):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of one outer iteration of the headline
    form, scaled by what the same counters read for the run's 4 GiB device-to-device copy
    (--calibrate-copy), averaged per kernel class -> profiles/traffic.json."""
    fetch, write = _counter_rows(fetch_dir), _counter_rows(write_dir)
    copy_bytes = 4.0 * 2**30

    def calib(rows):
        # the calibration copy is the program's first large device copy (--calibrate-copy
        # runs it before anything else)
        vals = [v for name, _, v in rows if "copyBuffer" in name and v * 1024.0 > 1e8]
        if not vals:
            raise SystemExit("no copy kernel in the counter record (run with --calibrate-copy)")
        return copy_bytes / (vals[0] * 1024.0)

    ff, wf = calib(fetch), calib(write)

    def per_kernel(rows, factor, prefix):
        # the runtime warm-up pair (200 nodes) dispatches the same kernels with tiny grids: keep the big ones
        vals = [(g, v) for name, g, v in rows if name.startswith(prefix)]
        if not vals:
            return None, 0
        gmax = max(g for g, _ in vals)
        big = [v for g, v in vals if g * 8 >= gmax]
        return sum(big) / len(big) * 1024.0 * factor, len(big)

    rec = dict(calibration=dict(fetch_factor=ff, write_factor=wf, reference="4 GiB device-to-device copy"),
               kernels={})
    lines = ["| kernel | launches | read GB/launch | written GB/launch | total GB/launch | algorithmic GB | ratio |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    import math as _m
    n = 120000
    chunk = n / _m.ceil(n / n_chunk(n, n, 4))
    for kind, prefix in KERNEL_NAMES.items():
        fb, nl = per_kernel(fetch, ff, prefix)
        wb, _ = per_kernel(write, wf, prefix)
        if fb is None or wb is None:
            continue
        alg = algorithmic_bytes(kind, n, n, 0, 0, chunk, 2, 6, transposed=False)  # the headline keeps no C^T
        rec["kernels"][kind] = dict(workload=workload, kernel=prefix, launches=nl, bytes_per_launch=fb + wb,
                                    fetch_bytes=fb, write_bytes=wb, algorithmic_bytes=alg,
                                    source_digest=source_digest(kind))
        lines.append(f"| `{prefix}` | {nl} | {fb / 1e9:.2f} | {wb / 1e9:.2f} | {(fb + wb) / 1e9:.2f} | "
                     f"{alg / 1e9:.2f} | {(fb + wb) / alg:.2f} |")
    with open(TRAFFIC, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"calibration: FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {wf:.4f}")
    print("\n".join(lines))


def main():
    args = parse()
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU in this build (asked for {args.gpus}); "
              "multi-GPU sharding is designed but not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2607_11952_amd import api, binding, warm
    from paper_2607_11952_amd.synth import CONFIGS, make_pair

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("torch and the device are up")
    if args.calibrate_copy:
        src = torch.empty(2**30, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        log("calibration copy: 4 GiB read + 4 GiB written")
    read_ceiling = measure_read_ceiling(api, torch, dev)
    log(f"streaming-read ceiling: {read_ceiling:.0f} GB/s")
    cfg = CONFIGS[args.workload]
    n1 = args.n or cfg.n1
    T = args.outer or cfg.outer_iters
    W, K = args.warmup, args.steps
    if K < 1 or W < 0:
        sys.exit("--steps must be >= 1 and --warmup >= 0")
    pair = make_pair(cfg, n1=n1)
    log(f"generated {cfg.name} n1={pair.n1} n2={pair.n2} m1={len(pair.edges1)} m2={len(pair.edges2)} "
        f"d={pair.X1.shape[1]} anchors={len(pair.anchors)}")
    inp = api.AlignInputs.from_pair(pair, dev)
    torch.cuda.synchronize()

    wpath = args.weights or warm.WEIGHTS
    mlp = None if args.cold else warm.load_weights(dev, wpath)
    common = dict(eps=cfg.eps, outer_iters=T, inner_iters=cfg.inner_iters, tol=1e-6, check_every=1, profile=1,
                  plan_in_ct=args.plan_in_ct)
    # top-2 lists of the final plan give each row's margin log(S_top / S_second)
    lean = dict(topk=10, dense_plan=False) if args.plan_in_ct else dict(topk=2)
    p_head = api.params(plan_dtype="bf16", feat_dtype="bf16", warm_start=mlp is not None, dual_start=args.start,
                        warm_probe=args.warm_probe, **common)
    p_plain = api.params(plan_dtype="f32", feat_dtype="f32", warm_start=False, dual_start="zero", **common)
    p_f32s = api.params(plan_dtype="f32", feat_dtype="f32", warm_start=False, dual_start=args.start, **common)

    # runtime warm-up on a tiny pair (loads the code objects; not a benchmark step)
    tiny = api.AlignInputs.from_pair(make_pair(CONFIGS["er1k"], n1=200), dev)
    api.align(tiny, api.params(outer_iters=1, inner_iters=2))
    torch.cuda.synchronize()

    truth = torch.from_numpy(pair.truth).to(dev).long()
    has_partner = truth >= 0
    # ranking test set (§4): true pairs that are not anchors
    test_truth = pair.truth.astype(np.int32).copy()
    test_truth[pair.anchors[:, 0]] = -1
    test_truth = torch.from_numpy(test_truth).to(dev)

    def ranking(rank):
        r = rank[rank > 0].double()
        return dict(hits_at_1=float((r <= 1).double().mean()), hits_at_10=float((r <= 10).double().mean()),
                    mrr=float((1.0 / r).mean()), test_pairs=int(r.numel()))

    def accuracy(am):
        """Share of the nodes of G1 with a true partner in G2 whose argmax is that partner."""
        return float((am.long()[has_partner] == truth[has_partner]).float().mean().item())

    def solve_summary(st, n_outer):
        n = min(n_outer, 64)
        return dict(inner_total=int(st.inner_total), marg_err_last=float(st.marg_err),
                    converged_all=bool(st.converged_all), inner_iters=[int(x) for x in list(st.inner_iters)[:n]],
                    inner_err=[float(x) for x in list(st.inner_err)[:n]],
                    warm=dict(fell_back=int(st.fell_back), warm_iters=int(st.warm_iters),
                              warm_err=float(st.warm_err), cold_iters=int(st.cold_iters),
                              cold_err=float(st.cold_err)))

    # ---------------- headline form: one alignment, its outer iterations are the steps
    al = api.Aligner(inp, p_head, mlp, test_truth, **lean)
    plan_gib = 0.0 if al.S is None else al.S.numel() * al.S.element_size() / 2**30
    log(f"headline form: workspace {al.ws_bytes / 2**30:.1f} GiB, plan {plan_gib:.1f} GiB, "
        f"warm start {mlp is not None}, later solves start {args.start}")
    n_outer = max(T, W + K)   # steps past T (only when W + K > T) continue the same iteration
    acc = binding.fa_stats()
    p1 = binding.fa_stats()
    torch.cuda.synchronize()
    e_all0, e_all1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e_k0, e_k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e_T = torch.cuda.Event(enable_timing=True)
    e_all0.record()
    al.begin(p1)
    for t in range(n_outer):
        if t == W:
            torch.cuda.synchronize()
            e_k0.record()
        al.step(t, last=(t == n_outer - 1), acc=acc if W <= t < W + K else None)
        if t == W + K - 1:
            e_k1.record()
            torch.cuda.synchronize()
            log(f"timed steps {W}..{W + K - 1}: {e_k0.elapsed_time(e_k1) / K / 1e3:.3f} s per outer iteration")
        if t == T - 1:
            e_T.record()
        if t < 3 or t % 10 == 9:
            log(f"outer iteration {t} done")
    res = al.end(n_outer)
    e_all1.record()
    torch.cuda.synchronize()
    ms_step = e_k0.elapsed_time(e_k1) / K
    align_ms = e_all0.elapsed_time(e_all1) if n_outer == T else e_all0.elapsed_time(e_T)
    head = dict(align_s=align_ms / 1e3, outer_iters_per_s=T / (align_ms / 1e3),
                ms_per_outer_timed=ms_step, **solve_summary(res.stats, n_outer),
                kernels_timed_steps=kernel_table(acc, pair, inp.A1.nnz, inp.A2.nnz, p_head, binding),
                phase_ms_timed_steps=dict(cost=acc.phase_ms[1], sinkhorn=acc.phase_ms[2], plan=acc.phase_ms[3]),
                phase1_ms=p1.phase_ms[0], kernels_phase1=kernel_table(p1, pair, inp.A1.nnz, inp.A2.nnz, p_head, binding),
                status=int(res.status))
    if n_outer != T:
        head["note"] = f"{n_outer} outer iterations ran; align_s covers Phase 1 and the first {T}"
    head["ranking"] = ranking(res.rank)
    head_argmax = res.argmax.clone()
    head_margin = margins(res)
    head["accuracy_vs_truth"] = accuracy(head_argmax)
    log(f"headline alignment: {align_ms / 1e3:.3f} s, inner iterations {res.stats.inner_total}, "
        f"last marginal error {res.stats.marg_err:.2e}, Hits@1 {head['ranking']['hits_at_1']:.4f}")
    del al, res
    torch.cuda.empty_cache()

    # ---------------- FP32 forms, one fa_align call each: the plain form (the paper's
    # method: cold starts) and, for the precision-only comparison, the headline's start
    # policy with an FP32 plan and operands (no learned start)
    skipped = []

    def full_run(name, p):
        est = 1.15 * align_ms / 1e3 + 15.0
        if time.time() - T_START + est > args.budget_s:
            skipped.append(f"{name} (needs ~{est:.0f} s, over the {args.budget_s:.0f} s budget)")
            return None, None
        al = api.Aligner(inp, p, None, test_truth, **lean)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        res = al.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out = dict(align_s=ms / 1e3, outer_iters_per_s=T / (ms / 1e3), **solve_summary(res.stats, T),
                   kernels=kernel_table(res.stats, pair, inp.A1.nnz, inp.A2.nnz, p, binding),
                   phase_ms=dict(phase1=res.stats.phase_ms[0], cost=res.stats.phase_ms[1],
                                 sinkhorn=res.stats.phase_ms[2], plan=res.stats.phase_ms[3]),
                   status=int(res.status), ranking=ranking(res.rank), accuracy_vs_truth=accuracy(res.argmax))
        out.update(agreement_with_headline(res.argmax, head_argmax, head_margin, margins(res)))
        log(f"{name}: {ms / 1e3:.3f} s, inner iterations {res.stats.inner_total}, last marginal error "
            f"{res.stats.marg_err:.2e}, argmax agreement with headline {out['argmax_agreement']:.4f}")
        del al, res
        torch.cuda.empty_cache()
        return out, out["argmax_agreement"]

    plain, agree = (None, None)
    if args.no_plain:
        skipped.append("plain (--no-plain)")
    else:
        plain, agree = full_run("plain FP32", p_plain)
    f32s = None
    if args.no_f32_mean or args.start == "zero":
        skipped.append("f32 with the headline start (--no-f32-mean or start zero)")
    else:
        f32s, _ = full_run(f"FP32, {args.start} start", p_f32s)

    # ---------------- roofline of the dominant kernel of the timed steps
    kt = head["kernels_timed_steps"]
    dom = max(kt.items(), key=lambda kv: kv[1]["total_ms"])
    ach = dom[1]["gbps"]
    wl = f"{cfg.name}:{pair.n1}x{pair.n2}"
    roofline = dict(bound="hbm", kernel=dom[0], achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                    traffic=measured_traffic(dom[0], wl), avg_ms=dom[1]["avg_ms"],
                    algorithmic_bytes_per_launch=dom[1]["algorithmic_bytes"],
                    read_ceiling_measured=read_ceiling, frac_of_read_ceiling=ach / read_ceiling)
    for k, v in kt.items():   # counter-measured HBM bytes per launch (None where stale or absent)
        mb = measured_traffic(k, wl)
        if mb is not None:
            v["hbm_bytes_measured"] = mb
            v["hbm_gbps_measured"] = mb / (v["avg_ms"] * 1e-3) / 1e9

    # ---------------- CPU baseline: the FP64 oracle on the host cores, bounded sample
    cpu = None
    if args.no_cpu:
        skipped.append("cpu_baseline (--no-cpu)")
    elif time.time() - T_START + 60.0 > args.budget_s:
        skipped.append("cpu_baseline (over the budget)")
    else:
        cpu = cpu_baseline(cfg, pair.n1, pair.n2, T, args.cpu_workers)

    spmm = {f"{form}_{k}": v["gbps"] for form, d in (("bf16", kt), ("f32", (plain or {}).get("kernels", {})))
            for k, v in d.items() if k.startswith("cost_stage")}
    line = dict(metric=METRIC, value=align_ms / 1e3, unit="s", n_gpus=1, steps=K, warmup=W,
                ms_per_step=ms_step, higher_is_better=False, scaling="weak", vs_baseline=None, dtype="bf16",
                data="synthetic",
                config=dict(workload=f"{cfg.name}: Chung-Lu n1={pair.n1} n2={pair.n2} avg_deg={cfg.avg_deg:g} "
                                     f"noise={cfg.noise:g} d={pair.X1.shape[1]} anchors={len(pair.anchors)} "
                                     f"eps={cfg.eps:g} outer={T} inner<={cfg.inner_iters} tol=1e-6",
                            n1=pair.n1, n2=pair.n2, outer_iters=T, inner_cap=cfg.inner_iters, tol=1e-6,
                            step="one outer iteration (cost rebuild + inner solve + plan) of the headline form",
                            value="device time of the whole headline alignment (Phase 1 + all outer iterations)"),
                warm_start=mlp is not None, warm_weights=os.path.relpath(wpath, ROOT) if mlp is not None else None,
                warm_probe=args.warm_probe, dual_start=args.start,
                plan_in_ct=args.plan_in_ct, headline=head,
                plain_fp32=plain, fp32_same_start=f32s, argmax_agreement=agree,
                speedup_vs_plain=(plain["align_s"] / head["align_s"] if plain else None),
                spmm_gbps=spmm, roofline=roofline, cpu_baseline=cpu, skipped=skipped,
                wall_s=time.time() - T_START)
    print(json.dumps(line), flush=True)


def margins(res):
    """Per row, log(S_top / S_second) of the final plan from its top-2 lists (None without them)."""
    import torch
    if res.topk_val is None or res.topk_val.shape[1] < 2:
        return None
    v = res.topk_val.double()
    return torch.log(v[:, 0] / v[:, 1].clamp_min(1e-300))


def agreement_with_headline(am, head_am, head_margin, margin):
    """Argmax agreement with the headline form, overall and on the rows that both plans
    resolve: top entry above the second by more than 1 and 4 nats in both."""
    out = dict(argmax_agreement=float((am == head_am).float().mean().item()))
    if margin is not None and head_margin is not None:
        for m in (1.0, 4.0):
            rows = (margin > m) & (head_margin > m)
            out[f"resolved_rows_{m:g}nat"] = float(rows.float().mean().item())
            out[f"agreement_on_resolved_{m:g}nat"] = float((am[rows] == head_am[rows]).float().mean().item())
    return out


def measure_read_ceiling(api, torch, dev, gib=32, reps=5):
    """Best of `reps` streaming reads of a `gib` GiB buffer (far larger than every cache)
    by the library's read kernel: the achievable read rate next to the 8 TB/s peak."""
    x = torch.ones(gib * 2**28, dtype=torch.float32, device=dev)
    nblk = 16384
    part = torch.empty(nblk * 256, dtype=torch.float32, device=dev)
    api.stream_read(x, part, nblk)
    best = math.inf
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        api.stream_read(x, part, nblk)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del x, part
    torch.cuda.empty_cache()
    return 4.0 * gib * 2**28 / (best * 1e-3) / 1e9


CPU_SAMPLE_N, CPU_SAMPLE_OUTER = 2500, 2


def _oracle_sample(cfg_name, seed_offset):
    """One oracle run on the bounded sample (a worker process; OMP/BLAS threads = 1)."""
    import numpy as np  # noqa: F401

    from oracle import fastalign_oracle as O
    from paper_2607_11952_amd.synth import CONFIGS, make_pair
    cfg = CONFIGS[cfg_name]
    pr = make_pair(cfg, n1=CPU_SAMPLE_N, seed=cfg.seed + seed_offset)
    rp1, ci1 = O.build_csr(pr.n1, pr.edges1)
    rp2, ci2 = O.build_csr(pr.n2, pr.edges2)
    p = O.Params(eps=cfg.eps, outer_iters=CPU_SAMPLE_OUTER, inner_iters=cfg.inner_iters, tol=1e-6)
    t0 = time.time()
    O.align(pr.n1, rp1, ci1, pr.n2, rp2, ci2, pr.X1, pr.X2, pr.anchors, p)
    return time.time() - t0, pr.n1, pr.n2


def cpu_baseline(cfg, n1_full, n2_full, T_full, workers=0):
    """The FP64 oracle as it stands, on every host core: one single-threaded oracle process
    per core, each aligning a sample pair of the same recipe (n = 2500, 2 outer iterations
    with the same inner cap and tolerance).  Throughput = samples / wall time; the full
    workload's time is extrapolated by n1 n2 and the outer-iteration count."""
    import multiprocessing as mp
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    P = workers if workers > 0 else min(cores, 16)
    env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    old = {k: os.environ.get(k) for k in env_keys}
    for k in env_keys:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")   # fresh interpreters that never touch the GPU
        t0 = time.time()
        with ctx.Pool(P) as pool:
            out = pool.starmap(_oracle_sample, [(cfg.name, 1000 + w) for w in range(P)])
        wall = time.time() - t0
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    per = [o[0] for o in out]
    ns1, ns2 = out[0][1], out[0][2]
    scale = (n1_full * n2_full) / (ns1 * ns2) * (T_full / CPU_SAMPLE_OUTER)
    # P samples finished in `wall` seconds of host time: the full workload is `scale` samples
    value = scale * wall / P
    log(f"oracle sample: {P} processes x n={ns1}, {CPU_SAMPLE_OUTER} outer, wall {wall:.1f}s "
        f"(per process {min(per):.1f}-{max(per):.1f}s) -> x{scale:.3g} / {P}")
    return dict(value=value, unit="s", cores=P, kind="oracle", extrapolated=True,
                sample=f"FP64 numpy/scipy oracle, {P} single-threaded processes in parallel (one per host core), "
                       f"each aligning a pair of the same recipe at n1={ns1} n2={ns2} for {CPU_SAMPLE_OUTER} outer x "
                       f"<= {cfg.inner_iters} inner iterations at tol 1e-6; wall {wall:.1f}s for {P} samples; "
                       f"value = wall/{P} x {scale:.4g} (n1*n2 and outer-count ratio to the workload)",
                sample_wall_s=wall, sample_per_process_s=per, host_cores_available=os.cpu_count())


if __name__ == "__main__":
    main()
