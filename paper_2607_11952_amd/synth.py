"""Seeded synthetic graph pairs for network alignment.

This module only builds inputs: edge lists, node features, anchor pairs and the
ground-truth correspondence. It contains none of the alignment arithmetic, so
both the GPU path and the CPU oracle may take their inputs from it.

The recipes stand in for the paper's workloads (two undirected graphs with node
attributes and a set of known anchor pairs, §2; Erdos-Renyi synthetics, §4.4):

* Erdos-Renyi G(n, p) and Chung-Lu power-law graphs (weights
  w_i ~ (i+1)^(-1/(gamma-1)), scaled to the average degree, capped at
  sqrt(sum w); endpoints drawn proportional to w; loops and duplicates dropped and
  topped up).
* G2 is a uniformly random relabelling of G1 with "x% edge noise": x% of the
  edges dropped uniformly and the same number of uniform non-edges added.
* Optionally G2 keeps only a uniformly chosen subset of its nodes (induced
  subgraph, relabelled in increasing order of the old label).
* Features: i.i.d. N(0,1) rows on G1; G2 gets the permuted copy plus N(0, sigma^2).
* Anchors: a uniform sample of the true pairs that survive in G2.

All randomness comes from numpy's PCG64 streams spawned from one SeedSequence.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = ["PairConfig", "GraphPair", "CONFIGS", "make_pair", "erdos_renyi",
           "chung_lu", "edge_noise"]


@dataclasses.dataclass(frozen=True)
class PairConfig:
    name: str
    n1: int
    kind: str = "er"            # "er" or "chung_lu"
    avg_deg: float = 8.0
    gamma: float = 2.5          # Chung-Lu degree exponent
    noise: float = 0.10         # fraction of edges dropped (and as many added)
    keep_n2: Optional[int] = None   # induced subgraph size of G2 (None: all nodes)
    d: int = 32
    sigma: float = 0.1
    anchor_frac: float = 0.10
    seed: int = 1
    # solver settings of the workload (not used by the generator itself)
    eps: float = 0.05
    outer_iters: int = 10
    inner_iters: int = 50


# The five workloads: a small parity case, a 20k power-law pair, an unequal-size
# pair for the reduced-precision form, the warm-start training family (template)
# and the largest single-GPU pair.
CONFIGS = {
    "er1k": PairConfig("er1k", 1000, "er", 8.0, noise=0.05, d=32, sigma=0.1,
                     anchor_frac=0.10, seed=1, eps=0.05, outer_iters=10, inner_iters=50),
    "cl20k": PairConfig("cl20k", 20000, "chung_lu", 12.0, noise=0.10, d=64, sigma=0.2,
                     anchor_frac=0.05, seed=2, eps=0.02, outer_iters=20, inner_iters=100),
    "cl60k_50k": PairConfig("cl60k_50k", 60000, "chung_lu", 16.0, noise=0.10, keep_n2=50000,
                     d=128, sigma=0.2, anchor_frac=0.05, seed=3, eps=0.02,
                     outer_iters=20, inner_iters=100),
    "warm_train": PairConfig("warm_train", 4000, "er", 12.0, noise=0.08, d=64, sigma=0.2,
                     anchor_frac=0.05, seed=1000, eps=0.02, outer_iters=20, inner_iters=100),
    "cl120k": PairConfig("cl120k", 120000, "chung_lu", 20.0, noise=0.10, d=128, sigma=0.2,
                     anchor_frac=0.02, seed=5, eps=0.02, outer_iters=30, inner_iters=100),
}


@dataclasses.dataclass
class GraphPair:
    n1: int
    n2: int
    edges1: np.ndarray      # int64 [m1, 2], undirected, each edge once
    edges2: np.ndarray      # int64 [m2, 2]
    X1: np.ndarray          # float32 [n1, d]
    X2: np.ndarray          # float32 [n2, d]
    anchors: np.ndarray     # int32 [nL, 2]  (node in G1, node in G2)
    truth: np.ndarray       # int64 [n1]: true partner in G2, or -1 if dropped
    config: Optional[PairConfig] = None


def _unique_pairs(u: np.ndarray, v: np.ndarray, n: int) -> np.ndarray:
    """Canonical (min, max) keys of the non-loop pairs, deduplicated."""
    keep = u != v
    a = np.minimum(u[keep], v[keep]).astype(np.int64)
    b = np.maximum(u[keep], v[keep]).astype(np.int64)
    return np.unique(a * n + b)


def erdos_renyi(n: int, avg_deg: float, rng: np.random.Generator) -> np.ndarray:
    """G(n, p) with p = avg_deg / (n - 1): Binomial edge count, uniform distinct pairs."""
    total = n * (n - 1) // 2
    p = min(1.0, avg_deg / max(n - 1, 1))
    m = int(rng.binomial(total, p)) if total > 0 else 0
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        draw = int(need * 1.1) + 16
        u = rng.integers(0, n, size=draw)
        v = rng.integers(0, n, size=draw)
        new = _unique_pairs(u, v, n)
        new = np.setdiff1d(new, keys, assume_unique=True)
        if new.size > need:
            new = rng.choice(new, size=need, replace=False)
        keys = np.union1d(keys, new)
    return np.stack([keys // n, keys % n], axis=1)


def chung_lu(n: int, avg_deg: float, gamma: float, rng: np.random.Generator) -> np.ndarray:
    """Chung-Lu power-law graph with m = n * avg_deg / 2 distinct edges."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    w *= n * avg_deg / w.sum()
    w = np.minimum(w, np.sqrt(w.sum()))
    prob = w / w.sum()
    cdf = np.cumsum(prob)
    cdf[-1] = 1.0
    m = int(round(n * avg_deg / 2))
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        draw = int(need * 1.2) + 16
        u = np.searchsorted(cdf, rng.random(draw), side="right")
        v = np.searchsorted(cdf, rng.random(draw), side="right")
        u = np.minimum(u, n - 1)
        v = np.minimum(v, n - 1)
        new = _unique_pairs(u, v, n)
        new = np.setdiff1d(new, keys, assume_unique=True)
        if new.size > need:
            new = rng.choice(new, size=need, replace=False)
        keys = np.union1d(keys, new)
    return np.stack([keys // n, keys % n], axis=1)


def edge_noise(edges: np.ndarray, n: int, frac: float, rng: np.random.Generator) -> np.ndarray:
    """Drop round(frac*m) edges uniformly, then add as many uniform non-edges."""
    m = edges.shape[0]
    k = int(round(frac * m))
    if k == 0 or m == 0:
        return edges.copy()
    keep = np.ones(m, dtype=bool)
    keep[rng.choice(m, size=k, replace=False)] = False
    kept = edges[keep]
    existing = np.minimum(edges[:, 0], edges[:, 1]) * n + np.maximum(edges[:, 0], edges[:, 1])
    existing = np.unique(existing)
    added = np.empty(0, dtype=np.int64)
    while added.size < k:
        need = k - added.size
        u = rng.integers(0, n, size=need * 2 + 16)
        v = rng.integers(0, n, size=need * 2 + 16)
        new = _unique_pairs(u, v, n)
        new = np.setdiff1d(new, existing, assume_unique=True)
        new = np.setdiff1d(new, added, assume_unique=True)
        if new.size > need:
            new = rng.choice(new, size=need, replace=False)
        added = np.union1d(added, new)
    add_e = np.stack([added // n, added % n], axis=1)
    return np.concatenate([kept, add_e], axis=0)


def make_pair(cfg: PairConfig, seed: Optional[int] = None, n1: Optional[int] = None) -> GraphPair:
    """Build the seeded graph pair described by ``cfg`` (seed / n1 may override)."""
    seed = cfg.seed if seed is None else seed
    n = cfg.n1 if n1 is None else n1
    ss = np.random.SeedSequence(seed)
    s_graph, s_relabel, s_perm, s_noise, s_keep, s_feat, s_anchor = ss.spawn(7)
    rg = np.random.Generator(np.random.PCG64(s_graph))
    if cfg.kind == "er":
        e = erdos_renyi(n, cfg.avg_deg, rg)
    elif cfg.kind == "chung_lu":
        e = chung_lu(n, cfg.avg_deg, cfg.gamma, rg)
    else:
        raise ValueError(f"unknown graph kind {cfg.kind!r}")
    # Random labels for G1 as well, so node ids carry no degree ordering.
    relabel = np.random.Generator(np.random.PCG64(s_relabel)).permutation(n)
    e1 = relabel[e]
    pi = np.random.Generator(np.random.PCG64(s_perm)).permutation(n)   # G1 node i -> G2 node pi[i]
    e2 = edge_noise(pi[e1], n, cfg.noise, np.random.Generator(np.random.PCG64(s_noise)))
    truth = pi.astype(np.int64)
    n2 = n
    if cfg.keep_n2 is not None and cfg.keep_n2 < n:
        keep_n = cfg.keep_n2 if n1 is None else int(round(n * cfg.keep_n2 / cfg.n1))
        kept = np.sort(np.random.Generator(np.random.PCG64(s_keep)).choice(n, size=keep_n, replace=False))
        newid = -np.ones(n, dtype=np.int64)
        newid[kept] = np.arange(keep_n)
        m2 = newid[e2]
        e2 = m2[(m2[:, 0] >= 0) & (m2[:, 1] >= 0)]
        truth = newid[pi]
        n2 = keep_n
    rf = np.random.Generator(np.random.PCG64(s_feat))
    X1 = rf.standard_normal((n, cfg.d)).astype(np.float32) if cfg.d > 0 else np.zeros((n, 0), np.float32)
    X2 = np.zeros((n2, cfg.d), dtype=np.float32)
    alive = truth >= 0
    if cfg.d > 0:
        X2[truth[alive]] = X1[alive] + cfg.sigma * rf.standard_normal((int(alive.sum()), cfg.d)).astype(np.float32)
    ra = np.random.Generator(np.random.PCG64(s_anchor))
    cand = np.nonzero(alive)[0]
    nL = int(round(cfg.anchor_frac * cand.size))
    pick = np.sort(ra.choice(cand, size=nL, replace=False)) if nL > 0 else np.empty(0, np.int64)
    anchors = np.stack([pick, truth[pick]], axis=1).astype(np.int32) if nL > 0 else np.zeros((0, 2), np.int32)
    return GraphPair(n1=n, n2=n2, edges1=e1.astype(np.int64), edges2=e2.astype(np.int64),
                     X1=X1, X2=X2, anchors=anchors, truth=truth, config=cfg)
