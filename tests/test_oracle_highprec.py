"""Pins of the oracle's Algorithm 1 that do not go through the oracle itself.

* The first outer iteration from S^0 = mu nu^T has a closed form: with a uniform
  plan, C1 S C2^T and Abar1^T S Abar2 are outer products of row sums of C1, C2
  and column sums of Abar1, Abar2 (Eq. (2), Algorithm 1, Phase 2), and the
  proximal term is + lambda_p log(n1 n2).
* Two four-node cases (a path against a path, a star against a path) evaluated
  with 50-digit arithmetic by explicit loops over the paper's definitions
  (§2.1-§2.3, Eqs. (1)-(4), Algorithm 1 with this repository's readings of the
  silent parts); the FP64 oracle must agree to 1e-12.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import fastalign_oracle as O
from paper_2607_11952_amd.synth import erdos_renyi


def _loop_adjacency(n, edges):
    A = np.zeros((n, n))
    for u, v in edges:
        if u != v:
            A[u, v] = A[v, u] = 1.0
    return A


def _ragged_pair(seed=5):
    r = np.random.default_rng(seed)
    n1, n2 = 9, 7
    e1 = erdos_renyi(n1, 3.0, r)
    e2 = erdos_renyi(n2, 2.5, r)
    X1 = r.standard_normal((n1, 3))
    X2 = r.standard_normal((n2, 3))
    L = np.array([[0, 2], [4, 5]])
    return n1, e1, n2, e2, X1, X2, L


def _first_cost_matches_closed_form(le, ln, la=0.6):
    n1, e1, n2, e2, X1, X2, L = _ragged_pair()
    p = O.Params(eps=0.2, lambda_e=le, lambda_n=ln, lambda_a=la, outer_iters=1, inner_iters=1, k_r=2)
    rp1, ci1 = O.build_csr(n1, e1)
    rp2, ci2 = O.build_csr(n2, e2)
    out = O.align(n1, rp1, ci1, n2, rp2, ci2, X1, X2, L, p, keep_history=True)
    C_first = out["history"][0]["C"]
    ph = out["phase1"]
    A1, A2 = _loop_adjacency(n1, e1), _loop_adjacency(n2, e2)
    d1, d2 = A1.sum(1), A2.sum(1)
    Ab1 = np.divide(A1, d1[:, None], out=np.zeros_like(A1), where=d1[:, None] > 0)
    Ab2 = np.divide(A2, d2[:, None], out=np.zeros_like(A2), where=d2[:, None] > 0)
    r1 = ph["C1"].toarray().sum(1)            # sum_k C1[i, k]
    r2 = ph["C2"].toarray().sum(1)            # sum_l C2[j, l]
    c1, c2 = Ab1.sum(0), Ab2.sum(0)           # sum_k Abar1[k, i], sum_l Abar2[l, j]
    N = float(n1 * n2)
    E = np.outer(r1, r2) / N
    P = np.outer(c1, c2) / N
    H = np.zeros((n1, n2))
    H[L[:, 0], L[:, 1]] = 1.0
    want = (ph["C_node"] + le * E - ln * np.log(P + p.delta_nbr) - la * np.log(p.ea + H)
            + p.lp * math.log(N))
    return np.allclose(C_first, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("le,ln", [(1.0, 0.0), (0.0, 1.0), (0.7, 1.3)])
def test_first_outer_iteration_from_the_uniform_plan(le, ln):
    """Cost of the first outer iteration = the closed form of Eq. (2) at S^0 = mu nu^T."""
    assert _first_cost_matches_closed_form(le, ln)


def test_first_outer_iteration_catches_a_wrong_initial_plan(monkeypatch):
    """The closed form above rejects S^0 = 1/n1 (a plan with the wrong mass)."""
    monkeypatch.setattr(O, "initial_log_plan", lambda n1, n2: np.full((n1, n2), -np.log(float(n1))))
    assert not _first_cost_matches_closed_form(1.0, 0.0)
    assert not _first_cost_matches_closed_form(0.0, 1.0)


# ---------------------------------------------------------------- 50 digits

mp.mp.dps = 50


def _mp_align(n1, edges1, n2, edges2, X1, X2, anchors, eps, alpha, beta, k_r, k_node, le, ln, la, T, K):
    """Algorithm 1 with 50-digit numbers and explicit loops, from the definitions:
    Abar = D^-1 A; R^(0) one-hot anchor columns, k_r steps R <- (1-beta) Abar R + beta R^(0);
    C_node = alpha e^{-R1 R2^T} + (1-alpha) e^{-Xh1 Xh2^T} (rows of X L2-normalised),
    then k_node steps C_node <- Abar1 C_node Abar2^T; C1 = (R1 R1^T) o Abar1,
    C2 = (R2 R2^T) o Abar2^T; C_anc = -log(eps + 1_L); S^0 = 1/(n1 n2); per outer
    iteration C = C_node + le C1 S C2^T - ln log(Abar1^T S Abar2 + delta) + la C_anc
    - eps log S, then K Sinkhorn iterations of Eq. (3) from a = b = 0 (a first), and
    S = exp((a_j + b_i - C_ij)/eps) (Eq. (4))."""
    f = mp.mpf

    def adj(n, edges):
        A = [[f(0)] * n for _ in range(n)]
        for u, v in edges:
            A[u][v] = A[v][u] = f(1)
        deg = [sum(row) for row in A]
        return [[A[i][k] / deg[i] if deg[i] > 0 else f(0) for k in range(n)] for i in range(n)]

    Ab1, Ab2 = adj(n1, edges1), adj(n2, edges2)
    nL = len(anchors)

    def encode(Ab, n, side):
        R0 = [[f(1) if anchors[l][side] == i else f(0) for l in range(nL)] for i in range(n)]
        R = [row[:] for row in R0]
        for _ in range(k_r):
            R = [[(1 - f(beta)) * sum(Ab[i][k] * R[k][l] for k in range(n)) + f(beta) * R0[i][l]
                  for l in range(nL)] for i in range(n)]
        return R

    R1, R2 = encode(Ab1, n1, 0), encode(Ab2, n2, 1)

    def normed(X):
        out = []
        for row in X:
            nr = mp.sqrt(sum(f(x) ** 2 for x in row))
            out.append([f(x) / nr if nr > 0 else f(0) for x in row])
        return out

    Xh1, Xh2 = normed(X1), normed(X2)
    dot = lambda u, v: sum(x * y for x, y in zip(u, v))
    Cn = [[f(alpha) * mp.exp(-dot(R1[i], R2[j])) + (1 - f(alpha)) * mp.exp(-dot(Xh1[i], Xh2[j]))
           for j in range(n2)] for i in range(n1)]
    for _ in range(k_node):
        Cn = [[sum(Ab1[i][k] * Cn[k][l] * Ab2[j][l] for k in range(n1) for l in range(n2))
               for j in range(n2)] for i in range(n1)]
    C1 = [[dot(R1[i], R1[k]) * Ab1[i][k] for k in range(n1)] for i in range(n1)]
    C2 = [[dot(R2[j], R2[l]) * Ab2[l][j] for l in range(n2)] for j in range(n2)]
    anc = {(int(u), int(v)) for u, v in anchors}
    Ca = [[-mp.log(f(eps) + (1 if (i, j) in anc else 0)) for j in range(n2)] for i in range(n1)]
    logS = [[-mp.log(f(n1 * n2))] * n2 for _ in range(n1)]
    S = [[mp.exp(x) for x in row] for row in logS]
    delta = f("1e-30")
    e = f(eps)
    for _ in range(T):
        C = [[None] * n2 for _ in range(n1)]
        for i in range(n1):
            for j in range(n2):
                E = sum(C1[i][k] * S[k][l] * C2[j][l] for k in range(n1) for l in range(n2))
                P = sum(Ab1[k][i] * S[k][l] * Ab2[l][j] for k in range(n1) for l in range(n2))
                C[i][j] = Cn[i][j] + le * E - ln * mp.log(P + delta) + la * Ca[i][j] - e * logS[i][j]
        a = [f(0)] * n2
        b = [f(0)] * n1
        for _ in range(K):
            a = [e * mp.log(f(1) / n2) - e * mp.log(sum(mp.exp((b[i] - C[i][j]) / e) for i in range(n1)))
                 for j in range(n2)]
            b = [e * mp.log(f(1) / n1) - e * mp.log(sum(mp.exp((a[j] - C[i][j]) / e) for j in range(n2)))
                 for i in range(n1)]
        logS = [[(a[j] + b[i] - C[i][j]) / e for j in range(n2)] for i in range(n1)]
        S = [[mp.exp(x) for x in row] for row in logS]
    return S, a, b


FOUR_NODE_CASES = {
    # path 0-1-2-3 against itself, one anchor at an end, 2-dim attributes
    "path-vs-path": (4, [(0, 1), (1, 2), (2, 3)], 4, [(0, 1), (1, 2), (2, 3)],
                     [[1.0, 0.2], [0.3, 1.0], [-0.5, 0.8], [0.9, -0.4]],
                     [[1.0, 0.3], [0.2, 1.1], [-0.6, 0.7], [0.8, -0.5]], [(0, 0)]),
    # star with centre 0 against the path 0-1-2-3, anchor centre <-> an inner node
    "star-vs-path": (4, [(0, 1), (0, 2), (0, 3)], 4, [(0, 1), (1, 2), (2, 3)],
                     [[0.5, 0.5], [1.0, -0.2], [0.1, 1.0], [-0.7, 0.3]],
                     [[0.9, -0.1], [0.4, 0.6], [0.2, 0.9], [-0.6, 0.4]], [(0, 1)]),
}


@pytest.mark.parametrize("case", sorted(FOUR_NODE_CASES))
def test_four_node_cases_against_fifty_digits(case):
    n1, e1, n2, e2, X1, X2, L = FOUR_NODE_CASES[case]
    kw = dict(eps=0.25, alpha=0.5, beta=0.15, k_r=3, k_node=1, le=1.0, ln=1.0, la=1.0, T=3, K=25)
    S_mp, a_mp, b_mp = _mp_align(n1, e1, n2, e2, X1, X2, L, **kw)
    S_ref = np.array([[float(x) for x in row] for row in S_mp])
    p = O.Params(eps=kw["eps"], alpha=kw["alpha"], beta=kw["beta"], k_r=kw["k_r"], k_node=kw["k_node"],
                 lambda_e=kw["le"], lambda_n=kw["ln"], lambda_a=kw["la"], outer_iters=kw["T"],
                 inner_iters=kw["K"])
    rp1, ci1 = O.build_csr(n1, np.array(e1))
    rp2, ci2 = O.build_csr(n2, np.array(e2))
    out = O.align(n1, rp1, ci1, n2, rp2, ci2, np.array(X1), np.array(X2), np.array(L), p)
    assert np.abs(out["S"] - S_ref).max() / S_ref.max() <= 1e-12
    assert np.abs(out["a"] - np.array([float(x) for x in a_mp])).max() <= 1e-12
    assert np.abs(out["b"] - np.array([float(x) for x in b_mp])).max() <= 1e-12
    assert list(out["argmax"]) == [int(np.argmax(r)) for r in S_ref]
    # the plan is a coupling of the uniform marginals up to the Sinkhorn residual
    assert np.allclose(S_ref.sum(1), 1.0 / n1, atol=1e-15)
