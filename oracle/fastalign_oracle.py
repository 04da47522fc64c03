"""FP64 CPU oracle of the FastAlign hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the graft
entry point and the CPU-baseline leg of the benchmark may import this module.
It shares no code with the GPU library: it takes plain numpy arrays, uses numpy
and scipy.sparse as its only primitives and never imports the product package.

Every function follows one step of the method as the paper states it:

* Problem statement and uniform marginals: §2.1, Eq. (1).
* Cost decomposition C = C_node + le*C_edge + ln*C_nbr + la*C_anc: §2.2, Eq. (2).
* Log-domain Sinkhorn dual updates: §2.3, Eq. (3).
* Plan recovery S = exp((a_j + b_i - C_ij)/eps): §2.3, Eq. (4).
* Linear-algebraic decomposition into Phase 1 (precompute), Phase 2 (S-dependent
  cost) and Phase 3 (Sinkhorn): §3.1, Algorithm 1.

Readings taken where the paper is silent or inconsistent (all of them are listed
with their reasons in the design notes of the repository):

* R1  Sinkhorn uses Eq. (3) with the log-marginal terms; the a-update (columns,
      paired with nu) runs before the b-update (rows, paired with mu).
* R2  Inner duals start at a = b = 0 at every outer iteration unless a start is
      given.
* R3  S^0 = mu nu^T (uniform).
* R4  The proximal term enters as  - lambda_p * log S  with log S carried as
      (a_j + b_i - C_prev_ij)/eps; lambda_p defaults to eps, so that
      exp(-C/eps) is the Gibbs kernel of the new cost times the previous plan.
* R5  A fixed number of outer iterations; the inner loop stops early only when
      tol > 0 and the L1 column-marginal violation after the b-update is <= tol.
* R6  Node-cost propagation is Abar1 @ C_node @ Abar2^T (neighbour average on
      both sides).
* R7  C2 = (R2 R2^T) * Abar2^T literally, i.e. C2[j,l] = (R2 R2^T)_jl / deg2_l.
* R8  C_nbr = -log(Abar1^T S Abar2 + delta) with delta = 1e-30.
* R9  The anchor cost uses its own eps_a (defaults to eps).
* R10 Features are row-L2-normalised before the similarity product (zero rows
      stay zero).
* R11 CSR: undirected, symmetrised, self-loops dropped, duplicates merged,
      columns sorted; isolated nodes have an all-zero normalised row.
* R12 argmax ties resolve to the lowest column index.
* R16 The top-k plan lists a row's k largest plan entries, larger log S first and,
      on equal log S, the lower column first (R12 extended to the whole list).
* R14 (variants) dual_start = "carry": every inner solve after the first starts
      from the final duals of the previous one instead of zeros; "mean": from the
      mean of the final duals of all earlier solves.  A solve run to convergence
      reaches the same optimum from any start (its duals are unique up to a
      constant shift that the plan and the cost update do not see), so the
      variants change only iterates that stop before convergence.
* R17 With the fallback on and tol > 0, a learned start (b_init) of the first
      solve gets warm_probe iterations (0: the full inner budget); if that solve
      misses tol, the solve is rerun from
      zero duals with the full budget, and the run keeps whichever of the two solves
      ends with the smaller marginal error (the cold start stays the reference).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Params", "build_csr", "row_normalized", "onehot_anchors", "positional_encoding",
    "l2_normalize_rows", "feature_similarity", "propagate", "anchor_cost", "intra_costs",
    "cost_update", "lse", "sinkhorn", "plan", "marginal_error", "initial_log_plan", "align",
    "similarity_entry", "propagate_entry", "intra_row_entries", "cost_entry", "row_dual_entry", "plan_entry",
    "true_partner_ranks", "hits_at_k", "mean_reciprocal_rank",
]


@dataclasses.dataclass
class Params:
    """Hyper-parameters of Algorithm 1 (the paper gives no values; these are ours)."""
    eps: float = 0.05
    alpha: float = 0.5
    beta: float = 0.15
    lambda_e: float = 1.0
    lambda_n: float = 1.0
    lambda_a: float = 1.0
    lambda_p: Optional[float] = None     # None -> eps
    eps_anchor: Optional[float] = None   # None -> eps
    delta_nbr: float = 1e-30
    tol: float = 0.0
    k_r: int = 10
    k_node: int = 1
    outer_iters: int = 10
    inner_iters: int = 50
    feat_l2norm: bool = True
    dual_start: str = "zero"             # R14: "zero", "carry" or "mean" start of the solves after the first
    warm_fallback: bool = True           # R17: rerun a learned start's solve cold when it misses tol
    warm_probe: int = 0                  # R17: iterations granted to the learned start (0: inner_iters)

    @property
    def lp(self) -> float:
        return self.eps if self.lambda_p is None else self.lambda_p

    @property
    def ea(self) -> float:
        return self.eps if self.eps_anchor is None else self.eps_anchor


# ----------------------------------------------------------------------------
# Graph input (§2: undirected graphs given by adjacency matrices)
# ----------------------------------------------------------------------------

def build_csr(n: int, edges: np.ndarray):
    """Symmetric pattern-only CSR of an undirected edge list (reading R11).

    Returns (rowptr int64[n+1], colidx int32[nnz]).  Raises ValueError on an
    endpoint outside [0, n).
    """
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if edges.size and (edges.min() < 0 or edges.max() >= n):
        raise ValueError("edge endpoint out of range")
    u, v = edges[:, 0], edges[:, 1]
    keep = u != v
    u, v = u[keep], v[keep]
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    key = np.unique(rows * n + cols)
    rows = key // n
    cols = key % n
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols.astype(np.int32)


def adjacency(n: int, rowptr: np.ndarray, colidx: np.ndarray) -> sp.csr_matrix:
    """0/1 adjacency matrix A as a scipy CSR matrix."""
    data = np.ones(colidx.shape[0], dtype=np.float64)
    return sp.csr_matrix((data, colidx.astype(np.int64), rowptr), shape=(n, n))


def row_normalized(n: int, rowptr: np.ndarray, colidx: np.ndarray):
    """Abar = D^-1 A (Algorithm 1, Phase 1: row normalisation); isolated rows stay 0.

    Returns (Abar as scipy CSR, deg float64[n]).
    """
    A = adjacency(n, rowptr, colidx)
    deg = np.asarray(A.sum(axis=1)).ravel()
    inv = np.zeros(n)
    inv[deg > 0] = 1.0 / deg[deg > 0]
    Abar = sp.diags(inv) @ A
    return sp.csr_matrix(Abar), deg


# ----------------------------------------------------------------------------
# Phase 1 (§3.1, Algorithm 1): S-independent quantities
# ----------------------------------------------------------------------------

def onehot_anchors(n: int, nodes: np.ndarray) -> np.ndarray:
    """R^(0): column l is one-hot at the anchor's node on this side."""
    nodes = np.asarray(nodes, dtype=np.int64)
    R0 = np.zeros((n, nodes.shape[0]))
    R0[nodes, np.arange(nodes.shape[0])] = 1.0
    return R0


def positional_encoding(Abar: sp.csr_matrix, R0: np.ndarray, beta: float, k: int) -> np.ndarray:
    """k steps of R <- (1-beta) Abar R + beta R^(0), starting from R^(0)."""
    R = R0.copy()
    for _ in range(k):
        R = (1.0 - beta) * (Abar @ R) + beta * R0
    return R


def l2_normalize_rows(X: np.ndarray) -> np.ndarray:
    """Row-wise L2 normalisation; zero rows stay zero (reading R10)."""
    X = np.asarray(X, dtype=np.float64)
    nrm = np.sqrt((X * X).sum(axis=1))
    out = np.zeros_like(X)
    nz = nrm > 0
    out[nz] = X[nz] / nrm[nz, None]
    return out


def feature_similarity(X1, X2, R1, R2, alpha: float, l2norm: bool = True) -> np.ndarray:
    """C_node = alpha * exp(-R1 R2^T) + (1 - alpha) * exp(-X1 X2^T), elementwise exp."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    if l2norm:
        X1 = l2_normalize_rows(X1)
        X2 = l2_normalize_rows(X2)
    return alpha * np.exp(-(R1 @ R2.T)) + (1.0 - alpha) * np.exp(-(X1 @ X2.T))


def propagate(Abar1: sp.csr_matrix, Abar2: sp.csr_matrix, C: np.ndarray, k: int) -> np.ndarray:
    """k steps of C <- Abar1 C Abar2^T (reading R6)."""
    for _ in range(k):
        left = Abar1 @ C                    # Abar1 C
        C = np.asarray((Abar2 @ left.T).T)  # (Abar1 C) Abar2^T
    return C


def anchor_cost(n1: int, n2: int, anchors: np.ndarray, eps_a: float) -> np.ndarray:
    """C_anc = -log(eps_a + OneHot(L)) as a dense matrix."""
    H = np.zeros((n1, n2))
    anchors = np.asarray(anchors, dtype=np.int64).reshape(-1, 2)
    H[anchors[:, 0], anchors[:, 1]] = 1.0
    return -np.log(eps_a + H)


def intra_costs(R1, Abar1: sp.csr_matrix, R2, Abar2: sp.csr_matrix):
    """C1 = (R1 R1^T) o Abar1 and C2 = (R2 R2^T) o Abar2^T, evaluated on the support only."""
    def sampled(R, M):
        M = sp.coo_matrix(M)
        vals = np.einsum("ij,ij->i", R[M.row], R[M.col]) * M.data
        return sp.csr_matrix((vals, (M.row, M.col)), shape=M.shape)
    return sampled(R1, Abar1), sampled(R2, sp.csr_matrix(Abar2.T))


# ----------------------------------------------------------------------------
# Phase 2 (§3.1, Algorithm 1; §2.2, Eq. (2)): S-dependent cost
# ----------------------------------------------------------------------------

def edge_cost(C1: sp.csr_matrix, C2: sp.csr_matrix, S: np.ndarray) -> np.ndarray:
    """C_edge = C1 S C2^T."""
    left = C1 @ S
    return np.asarray((C2 @ left.T).T)


def nbr_product(Abar1: sp.csr_matrix, Abar2: sp.csr_matrix, S: np.ndarray) -> np.ndarray:
    """Abar1^T S Abar2 (the argument of the neighbourhood cost's log)."""
    left = Abar1.T @ S
    return np.asarray((Abar2.T @ left.T).T)


def cost_update(C_node, C_anc, C1, C2, Abar1, Abar2, S, logS, p: Params) -> np.ndarray:
    """C = C_node + le*C1 S C2^T - ln*log(Abar1^T S Abar2 + delta) + la*C_anc - lp*log S."""
    E = edge_cost(C1, C2, S)
    P = nbr_product(Abar1, Abar2, S)
    return (C_node + p.lambda_e * E - p.lambda_n * np.log(P + p.delta_nbr)
            + p.lambda_a * C_anc - p.lp * logS)


# ----------------------------------------------------------------------------
# Phase 3 (§2.3, Eqs. (3)-(4)): log-domain Sinkhorn and the plan
# ----------------------------------------------------------------------------

def lse(x: np.ndarray, axis: int) -> np.ndarray:
    """log-sum-exp with the max shift: m + log(sum(exp(x - m)))."""
    m = np.max(x, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    out = m + np.log(np.sum(np.exp(x - m), axis=axis, keepdims=True))
    return np.squeeze(out, axis=axis)


def plan(C: np.ndarray, a: np.ndarray, b: np.ndarray, eps: float) -> np.ndarray:
    """S_ij = exp((a_j + b_i - C_ij)/eps), Eq. (4)."""
    return np.exp((a[None, :] + b[:, None] - C) / eps)


def plan_topk(C: np.ndarray, a: np.ndarray, b: np.ndarray, eps: float, k: int):
    """Per row the k largest entries of the plan of Eq. (4) and their columns (R16).

    The plan is concentrated on few entries per row (§3.3, memory reduction); the
    list is the plan restricted to them.  Returns (values [n1, k], columns [n1, k]).
    """
    logS = (a[None, :] + b[:, None] - C) / eps
    n1, n2 = logS.shape
    cols = np.broadcast_to(np.arange(n2), (n1, n2))
    order = np.lexsort((cols, -logS), axis=1)[:, :k]   # primary: log S descending; then column
    return np.exp(np.take_along_axis(logS, order, axis=1)), order


def marginal_error(C, a, b, eps: float) -> float:
    """L1 violation of the column marginal nu = 1/n2 by the plan of (a, b)."""
    n2 = C.shape[1]
    return float(np.abs(plan(C, a, b, eps).sum(axis=0) - 1.0 / n2).sum())


def sinkhorn(C: np.ndarray, eps: float, n_iter: int, tol: float = 0.0,
             a0: Optional[np.ndarray] = None, b0: Optional[np.ndarray] = None):
    """Eq. (3): alternate a-updates (over rows i, per column j) and b-updates.

    Returns (a, b, iterations_done, marginal_error_after_last_b_update).
    """
    n1, n2 = C.shape
    log_mu = np.log(1.0 / n1)
    log_nu = np.log(1.0 / n2)
    a = np.zeros(n2) if a0 is None else np.array(a0, dtype=np.float64)
    b = np.zeros(n1) if b0 is None else np.array(b0, dtype=np.float64)
    err = marginal_error(C, a, b, eps)
    it = 0
    while it < n_iter:
        a = eps * log_nu - eps * lse((b[:, None] - C) / eps, axis=0)
        b = eps * log_mu - eps * lse((a[None, :] - C) / eps, axis=1)
        it += 1
        err = marginal_error(C, a, b, eps)
        if tol > 0 and err <= tol:
            break
    return a, b, it, err


# ----------------------------------------------------------------------------
# Algorithm 1 end to end
# ----------------------------------------------------------------------------

def phase1(n1, rowptr1, colidx1, n2, rowptr2, colidx2, X1, X2, anchors, p: Params):
    """All S-independent quantities of Algorithm 1, Phase 1."""
    anchors = np.asarray(anchors, dtype=np.int64).reshape(-1, 2)
    Abar1, deg1 = row_normalized(n1, rowptr1, colidx1)
    Abar2, deg2 = row_normalized(n2, rowptr2, colidx2)
    R1 = positional_encoding(Abar1, onehot_anchors(n1, anchors[:, 0]), p.beta, p.k_r)
    R2 = positional_encoding(Abar2, onehot_anchors(n2, anchors[:, 1]), p.beta, p.k_r)
    X1 = np.asarray(X1, dtype=np.float64).reshape(n1, -1)
    X2 = np.asarray(X2, dtype=np.float64).reshape(n2, -1)
    C_node = feature_similarity(X1, X2, R1, R2, p.alpha, p.feat_l2norm)
    C_node = propagate(Abar1, Abar2, C_node, p.k_node)
    C_anc = anchor_cost(n1, n2, anchors, p.ea)
    C1, C2 = intra_costs(R1, Abar1, R2, Abar2)
    return dict(Abar1=Abar1, Abar2=Abar2, deg1=deg1, deg2=deg2, R1=R1, R2=R2,
                C_node=C_node, C_anc=C_anc, C1=C1, C2=C2)


def initial_log_plan(n1: int, n2: int) -> np.ndarray:
    """log S^0 for S^0 = mu nu^T with the uniform marginals of Eq. (1) (reading R3)."""
    return np.full((n1, n2), -np.log(float(n1) * float(n2)))


def align(n1, rowptr1, colidx1, n2, rowptr2, colidx2, X1, X2, anchors, p: Params,
          b_init: Optional[np.ndarray] = None, keep_history: bool = False):
    """Algorithm 1: Phase 1 once, then outer iterations of Phase 2 + Phase 3.

    ``b_init`` (optional) replaces the zero row duals of the first outer solve.
    Returns a dict with S, a, b, argmax, the last cost C, per-outer inner
    iteration counts and marginal errors.
    """
    if p.dual_start not in ("zero", "carry", "mean"):
        raise ValueError(f"unknown dual_start {p.dual_start!r}")
    ph = phase1(n1, rowptr1, colidx1, n2, rowptr2, colidx2, X1, X2, anchors, p)
    logS = initial_log_plan(n1, n2)
    S = np.exp(logS)
    iters, errs, hist = [], [], []
    a = np.zeros(n2)
    b = np.zeros(n1)
    solved_a, solved_b = [], []
    warm = dict(warm_iters=-1, warm_err=float("nan"), cold_iters=-1, cold_err=float("nan"), fell_back=0)
    C = None
    for t in range(p.outer_iters):
        C = cost_update(ph["C_node"], ph["C_anc"], ph["C1"], ph["C2"], ph["Abar1"],
                        ph["Abar2"], S, logS, p)
        a0 = b0 = None                      # zero start
        if t == 0 and b_init is not None:
            b0 = b_init
        elif t > 0 and p.dual_start == "carry":
            a0, b0 = a, b
        elif t > 0 and p.dual_start == "mean":
            a0 = sum(solved_a) / len(solved_a)
            b0 = sum(solved_b) / len(solved_b)
        budget = p.inner_iters
        if t == 0 and b_init is not None and p.warm_fallback and p.tol > 0 and p.warm_probe > 0:
            budget = min(p.warm_probe, p.inner_iters)
        a, b, it, err = sinkhorn(C, p.eps, budget, p.tol, a0, b0)
        if t == 0 and b_init is not None:
            warm.update(warm_iters=it, warm_err=err)
            if p.warm_fallback and p.tol > 0 and not err <= p.tol:
                ac, bc, itc, errc = sinkhorn(C, p.eps, p.inner_iters, p.tol)
                warm.update(cold_iters=itc, cold_err=errc)
                if errc < err:
                    a, b, err = ac, bc, errc
                    warm["fell_back"] = 2
                it += itc
        solved_a.append(a)
        solved_b.append(b)
        logS = (a[None, :] + b[:, None] - C) / p.eps
        S = np.exp(logS)
        iters.append(it)
        errs.append(err)
        if keep_history:
            hist.append(dict(C=C.copy(), a=a.copy(), b=b.copy()))
    argmax = np.argmax(S, axis=1) if n2 > 0 else np.zeros(n1, dtype=np.int64)
    return dict(S=S, a=a, b=b, argmax=argmax, C=C, iters=iters, errs=errs,
                phase1=ph, history=hist, **warm)


# ----------------------------------------------------------------------------
# Single entries, for sampled checks at sizes where the dense matrices above do
# not fit in host memory.  Each is the definition above evaluated at one (i, j)
# from the few operand entries it depends on.
# ----------------------------------------------------------------------------

def similarity_entry(x1, x2, r1, r2, alpha: float) -> float:
    """C_node[i, j] (Phase 1) from row i of X1, R1 and row j of X2, R2 (already normalised)."""
    x1, x2, r1, r2 = (np.asarray(v, dtype=np.float64) for v in (x1, x2, r1, r2))
    return float(alpha * np.exp(-(r1 @ r2)) + (1.0 - alpha) * np.exp(-(x1 @ x2)))


def propagate_entry(C_block, deg1_i: int, deg2_j: int) -> float:
    """(Abar1 C Abar2^T)[i, j] with C_block = C[N1(i)][:, N2(j)]; every entry of row i
    of Abar1 is 1/deg1(i) and of row j of Abar2 is 1/deg2(j)."""
    if deg1_i == 0 or deg2_j == 0:
        return 0.0
    return float(np.asarray(C_block, dtype=np.float64).sum() / (float(deg1_i) * float(deg2_j)))


def intra_row_entries(r_i, R_nbrs, scale) -> np.ndarray:
    """Entries of C1 (or C2) on one row's support: (R R^T)[i, k] * scale, scale being the
    Abar factor (1/deg1(i) for C1 = (R1R1^T) o Abar1; 1/deg2(l) per neighbour l for
    C2 = (R2R2^T) o Abar2^T)."""
    return (np.asarray(R_nbrs, dtype=np.float64) @ np.asarray(r_i, dtype=np.float64)) * np.asarray(scale,
                                                                                                  dtype=np.float64)


def cost_entry(S_block, c1_row, c2_row, inv1_nbr, inv2_nbr, c_node: float, anchored: bool,
               logS_prev: float, p: Params) -> float:
    """Eq. (2) plus the proximal term at one (i, j), with
    S_block = S[N1(i)][:, N2(j)], c1_row[k] = C1[i, N1(i)_k], c2_row[l] = C2[j, N2(j)_l],
    inv1_nbr[k] = Abar1[N1(i)_k, i] = 1/deg1(N1(i)_k), inv2_nbr[l] = Abar2[N2(j)_l, j]."""
    S_block = np.asarray(S_block, dtype=np.float64)
    E = float(np.asarray(c1_row, dtype=np.float64) @ S_block @ np.asarray(c2_row, dtype=np.float64))
    P = float(np.asarray(inv1_nbr, dtype=np.float64) @ S_block @ np.asarray(inv2_nbr, dtype=np.float64))
    anc = -np.log(p.ea + (1.0 if anchored else 0.0))
    return float(c_node + p.lambda_e * E - p.lambda_n * np.log(P + p.delta_nbr) + p.lambda_a * anc
                 - p.lp * logS_prev)


def row_dual_entry(c_row, a, eps: float, n1: int) -> float:
    """The b-update of Eq. (3) for one row i: eps log mu_i - eps LSE_j((a_j - C_ij)/eps)."""
    x = (np.asarray(a, dtype=np.float64) - np.asarray(c_row, dtype=np.float64)) / eps
    return float(eps * np.log(1.0 / n1) - eps * lse(x, axis=0))


def plan_entry(c: float, a_j: float, b_i: float, eps: float) -> float:
    """Eq. (4) at one (i, j)."""
    return float(np.exp((a_j + b_i - c) / eps))


# ----------------------------------------------------------------------------
# Ranking readout of §4: Hits@K and MRR over the true partners
# ----------------------------------------------------------------------------

def true_partner_ranks(scores: np.ndarray, truth: np.ndarray) -> np.ndarray:
    """Per row i with a true partner t = truth[i] in [0, n2): the rank of t among the
    row's alignment scores, 1 + #{j : scores[i, j] > scores[i, t]}; 0 for other rows."""
    scores = np.asarray(scores, dtype=np.float64)
    n1, n2 = scores.shape
    truth = np.asarray(truth, dtype=np.int64)
    ranks = np.zeros(n1, dtype=np.int64)
    for i in range(n1):
        t = truth[i]
        if 0 <= t < n2:
            ranks[i] = 1 + int(np.count_nonzero(scores[i] > scores[i, t]))
    return ranks


def hits_at_k(ranks: np.ndarray, k: int) -> float:
    """Share of the ranked rows (rank > 0) whose true partner is among the top k."""
    r = np.asarray(ranks)
    r = r[r > 0]
    return float(np.mean(r <= k)) if r.size else 0.0


def mean_reciprocal_rank(ranks: np.ndarray) -> float:
    r = np.asarray(ranks, dtype=np.float64)
    r = r[r > 0]
    return float(np.mean(1.0 / r)) if r.size else 0.0
