"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test fixes one step with something independent: a closed form, an
invariant of the mathematics, a brute-force evaluation with explicit loops on a
tiny input, or a textbook/library routine for a special case.  A plausible slip
in the oracle (dropped term, wrong sign, transposed operand, swapped dual)
breaks at least one of them; ``test_planted_mistakes_are_caught`` checks that
claim for a few such slips.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

from oracle import fastalign_oracle as O
from paper_2607_11952_amd.synth import CONFIGS, make_pair, erdos_renyi


def rng(seed=0):
    return np.random.default_rng(seed)


def tiny_graph(n, m, seed, loops=True):
    r = rng(seed)
    e = r.integers(0, n, size=(m, 2))
    if not loops:
        e = e[e[:, 0] != e[:, 1]]
    return e


def dense_adj_loops(n, edges):
    """Adjacency by explicit loops: undirected, no self-loops, 0/1."""
    A = np.zeros((n, n))
    for u, v in edges:
        if u != v:
            A[u, v] = 1.0
            A[v, u] = 1.0
    return A


# ---------------------------------------------------------------- graph input

@pytest.mark.parametrize("seed", range(5))
def test_csr_matches_loop_built_adjacency(seed):
    n = 9
    edges = tiny_graph(n, 30, seed)
    rp, ci = O.build_csr(n, edges)
    A = dense_adj_loops(n, edges)
    # dense round trip
    D = np.zeros((n, n))
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            D[i, ci[e]] += 1.0
    assert np.array_equal(D, A)
    # sorted, no duplicates, no loops
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
        assert i not in row
    assert rp.dtype == np.int64 and ci.dtype == np.int32


def test_csr_isolated_and_empty():
    rp, ci = O.build_csr(4, np.zeros((0, 2), np.int64))
    assert np.array_equal(rp, np.zeros(5, np.int64)) and ci.size == 0
    rp, ci = O.build_csr(4, np.array([[1, 1], [2, 3], [3, 2]]))
    assert list(rp) == [0, 0, 0, 1, 2] and list(ci) == [3, 2]
    with pytest.raises(ValueError):
        O.build_csr(3, np.array([[0, 3]]))


def test_row_normalized_rows_sum_to_one():
    n = 12
    rp, ci = O.build_csr(n, tiny_graph(n, 10, 3))
    Abar, deg = O.row_normalized(n, rp, ci)
    rs = np.asarray(Abar.sum(axis=1)).ravel()
    for i in range(n):
        if deg[i] > 0:
            assert abs(rs[i] - 1.0) < 1e-15
        else:
            assert rs[i] == 0.0
    assert (deg == 0).any()  # the case covers isolated nodes


# ---------------------------------------------------------------- Phase 1

def test_positional_encoding_closed_form():
    n, beta, k = 10, 0.3, 6
    rp, ci = O.build_csr(n, tiny_graph(n, 18, 4))
    Abar, _ = O.row_normalized(n, rp, ci)
    R0 = O.onehot_anchors(n, np.array([1, 4, 7]))
    R = O.positional_encoding(Abar, R0, beta, k)
    M = Abar.toarray()
    mp = np.linalg.matrix_power
    closed = (1 - beta) ** k * mp(M, k) @ R0 + beta * sum((1 - beta) ** t * mp(M, t) @ R0 for t in range(k))
    assert np.allclose(R, closed, rtol=0, atol=1e-14)
    # one-hot structure of R^(0)
    assert np.array_equal(R0.sum(axis=0), np.ones(3)) and R0[4, 1] == 1.0


def test_feature_similarity_elementwise_loops():
    r = rng(5)
    n1, n2, d, L = 4, 5, 3, 2
    X1, X2 = r.standard_normal((n1, d)), r.standard_normal((n2, d))
    X1[2] = 0.0  # a zero feature row stays zero after normalisation
    R1, R2 = r.random((n1, L)), r.random((n2, L))
    alpha = 0.3
    C = O.feature_similarity(X1, X2, R1, R2, alpha, l2norm=True)
    for i in range(n1):
        for j in range(n2):
            n_i = math.sqrt(sum(x * x for x in X1[i]))
            n_j = math.sqrt(sum(x * x for x in X2[j]))
            cos = 0.0 if n_i == 0 else sum(X1[i, q] * X2[j, q] for q in range(d)) / (n_i * n_j)
            rr = sum(R1[i, q] * R2[j, q] for q in range(L))
            want = alpha * math.exp(-rr) + (1 - alpha) * math.exp(-cos)
            assert abs(C[i, j] - want) < 1e-14
    # alpha = 1 drops the feature term, alpha = 0 drops the positional term
    assert np.allclose(O.feature_similarity(X1, X2, R1, R2, 1.0), np.exp(-(R1 @ R2.T)), atol=0)


def test_propagate_brute_force_and_constant():
    n1, n2 = 7, 6
    rp1, ci1 = O.build_csr(n1, tiny_graph(n1, 12, 6))
    rp2, ci2 = O.build_csr(n2, tiny_graph(n2, 10, 7))
    A1, d1 = O.row_normalized(n1, rp1, ci1)
    A2, d2 = O.row_normalized(n2, rp2, ci2)
    C = rng(8).random((n1, n2))
    got = O.propagate(A1, A2, C, 1)
    M1, M2 = A1.toarray(), A2.toarray()
    want = np.zeros((n1, n2))
    for i in range(n1):
        for j in range(n2):
            want[i, j] = sum(M1[i, k] * C[k, l] * M2[j, l] for k in range(n1) for l in range(n2))
    assert np.allclose(got, want, atol=1e-15)
    # a neighbour average keeps a constant where both nodes have neighbours
    K = O.propagate(A1, A2, np.full((n1, n2), 2.5), 2)
    mask = (d1[:, None] > 0) & (d2[None, :] > 0)
    assert np.allclose(K[mask], 2.5, atol=1e-15) and np.all(K[~mask] == 0)


def test_anchor_cost_values():
    C = O.anchor_cost(3, 4, np.array([[0, 2], [2, 1]]), 0.05)
    assert C[0, 2] == pytest.approx(-math.log(1.05)) and C[2, 1] == pytest.approx(-math.log(1.05))
    assert C[1, 1] == pytest.approx(-math.log(0.05))
    assert (C == -math.log(0.05)).sum() == 10


def test_intra_costs_dense_mask():
    n1, n2, L = 8, 7, 3
    rp1, ci1 = O.build_csr(n1, tiny_graph(n1, 14, 9))
    rp2, ci2 = O.build_csr(n2, tiny_graph(n2, 12, 10))
    A1, _ = O.row_normalized(n1, rp1, ci1)
    A2, _ = O.row_normalized(n2, rp2, ci2)
    R1, R2 = rng(11).random((n1, L)), rng(12).random((n2, L))
    C1, C2 = O.intra_costs(R1, A1, R2, A2)
    assert np.allclose(C1.toarray(), (R1 @ R1.T) * A1.toarray(), atol=1e-15)
    assert np.allclose(C2.toarray(), (R2 @ R2.T) * A2.toarray().T, atol=1e-15)


# ---------------------------------------------------------------- Phase 2

def test_cost_terms_brute_force():
    n1, n2, L = 6, 5, 2
    rp1, ci1 = O.build_csr(n1, tiny_graph(n1, 10, 13))
    rp2, ci2 = O.build_csr(n2, tiny_graph(n2, 9, 14))
    A1, _ = O.row_normalized(n1, rp1, ci1)
    A2, _ = O.row_normalized(n2, rp2, ci2)
    R1, R2 = rng(15).random((n1, L)), rng(16).random((n2, L))
    C1, C2 = O.intra_costs(R1, A1, R2, A2)
    S = rng(17).random((n1, n2))
    M1, M2, K1, K2 = A1.toarray(), A2.toarray(), C1.toarray(), C2.toarray()
    E = np.zeros((n1, n2))
    P = np.zeros((n1, n2))
    for i in range(n1):
        for j in range(n2):
            E[i, j] = sum(K1[i, k] * S[k, l] * K2[j, l] for k in range(n1) for l in range(n2))
            P[i, j] = sum(M1[k, i] * S[k, l] * M2[l, j] for k in range(n1) for l in range(n2))
    assert np.allclose(O.edge_cost(C1, C2, S), E, atol=1e-15)
    assert np.allclose(O.nbr_product(A1, A2, S), P, atol=1e-15)
    p = O.Params(eps=0.1, lambda_e=0.7, lambda_n=1.3, lambda_a=0.4, lambda_p=0.2)
    Cn, Ca = rng(18).random((n1, n2)), rng(19).random((n1, n2))
    logS = np.log(S)
    got = O.cost_update(Cn, Ca, C1, C2, A1, A2, S, logS, p)
    want = Cn + 0.7 * E - 1.3 * np.log(P + 1e-30) + 0.4 * Ca - 0.2 * logS
    assert np.allclose(got, want, atol=1e-13)


def test_nbr_product_conserves_mass():
    # With no isolated node, every column of Abar1 and Abar2 rows is a distribution:
    # sum(Abar1^T S Abar2) = 1^T Abar1^T S Abar2 1 = (Abar1 1)^T S (Abar2 1) = sum(S).
    pr = make_pair(CONFIGS["er1k"])
    rp1, ci1 = O.build_csr(pr.n1, pr.edges1)
    deg = np.diff(rp1)
    if (deg == 0).any():
        pytest.skip("graph has isolated nodes")
    A1, _ = O.row_normalized(pr.n1, rp1, ci1)
    S = rng(20).random((pr.n1, 300))
    n2 = 300
    e2 = erdos_renyi(n2, 10, rng(21))
    rp2, ci2 = O.build_csr(n2, e2)
    if (np.diff(rp2) == 0).any():
        pytest.skip("graph has isolated nodes")
    A2, _ = O.row_normalized(n2, rp2, ci2)
    P = O.nbr_product(A1, A2, S)
    assert abs(P.sum() - S.sum()) < 1e-9 * S.sum()


# ---------------------------------------------------------------- Phase 3

def test_sinkhorn_zero_and_additive_cost():
    n1, n2, eps = 5, 7, 0.1
    for C in (np.zeros((n1, n2)), np.add.outer(rng(22).random(n1) * 3, rng(23).random(n2) * 2)):
        a, b, it, err = O.sinkhorn(C, eps, 1)
        S = O.plan(C, a, b, eps)
        assert np.allclose(S, np.full((n1, n2), 1.0 / (n1 * n2)), rtol=1e-13, atol=0)
        assert err < 1e-14


@pytest.mark.parametrize("delta,eps", [(0.3, 0.1), (-1.0, 0.25), (2.0, 0.5)])
def test_sinkhorn_two_by_two_closed_form(delta, eps):
    C = np.array([[delta, 0.0], [0.0, 0.0]])
    a, b, it, err = O.sinkhorn(C, eps, 2000, tol=1e-15)
    S = O.plan(C, a, b, eps)
    x = 1.0 / (2.0 * (1.0 + math.exp(delta / (2 * eps))))
    assert np.allclose(S, [[x, 0.5 - x], [0.5 - x, x]], atol=1e-13)


def test_sinkhorn_marginals_to_1e10_and_matches_matrix_scaling():
    r = rng(24)
    n1, n2, eps = 30, 20, 0.2
    C = r.random((n1, n2))
    a, b, it, err = O.sinkhorn(C, eps, 10000, tol=1e-12)
    S = O.plan(C, a, b, eps)
    assert np.abs(S.sum(axis=0) - 1 / n2).sum() <= 1e-10
    assert np.abs(S.sum(axis=1) - 1 / n1).sum() <= 1e-10
    # textbook matrix scaling u = mu / (K v), v = nu / (K^T u) in the primal domain
    K = np.exp(-C / eps)
    u, v = np.ones(n1), np.ones(n2)
    for _ in range(20000):
        v = (1 / n2) / (K.T @ u)
        u = (1 / n1) / (K @ v)
    assert np.allclose(S, u[:, None] * K * v[None, :], rtol=1e-9, atol=0)


def test_sinkhorn_solves_entropic_ot_directly():
    """Eq. (1) solved by a generic constrained optimiser on a 3x3 problem."""
    r = rng(25)
    n, eps = 3, 0.3
    C = r.random((n, n))
    mu = np.full(n, 1 / n)

    def f(x):
        S = x.reshape(n, n)
        return float((S * C).sum() + eps * (S * (np.log(S) - 1)).sum())

    cons = [{"type": "eq", "fun": lambda x, i=i: x.reshape(n, n)[i].sum() - mu[i]} for i in range(n)]
    cons += [{"type": "eq", "fun": lambda x, j=j: x.reshape(n, n)[:, j].sum() - mu[j]} for j in range(n - 1)]
    res = so.minimize(f, np.full(n * n, 1 / n ** 2), method="SLSQP", constraints=cons,
                      bounds=[(1e-12, 1)] * (n * n), options=dict(ftol=1e-15, maxiter=1000))
    a, b, _, _ = O.sinkhorn(C, eps, 5000, tol=1e-14)
    assert np.allclose(O.plan(C, a, b, eps), res.x.reshape(n, n), atol=2e-6)


def test_sinkhorn_invariants_cross_ratio_and_monotone_dual():
    r = rng(26)
    n1, n2, eps = 6, 8, 0.15
    C = r.random((n1, n2)) * 2
    mu, nu = 1 / n1, 1 / n2

    def dual(a, b):
        return nu * a.sum() + mu * b.sum() - eps * np.exp((a[None, :] + b[:, None] - C) / eps).sum()

    K = np.exp(-C / eps)
    a, b = np.zeros(n2), np.zeros(n1)
    prev = dual(a, b)
    for _ in range(30):
        a, b, _, _ = O.sinkhorn(C, eps, 1, 0, a, b)
        S = O.plan(C, a, b, eps)
        cr = S[0, 1] * S[2, 3] / (S[0, 3] * S[2, 1])
        assert cr == pytest.approx(K[0, 1] * K[2, 3] / (K[0, 3] * K[2, 1]), rel=1e-12)
        cur = dual(a, b)
        assert cur >= prev - 1e-15
        prev = cur


def test_lse_large_magnitudes_and_single_element():
    x = np.array([[1000.0, 1000.0, 1000.0], [-1e3, -1e3 + math.log(2), -np.inf]])
    out = O.lse(x, axis=1)
    assert out[0] == pytest.approx(1000 + math.log(3), abs=1e-12)
    assert out[1] == pytest.approx(-1e3 + math.log(3), abs=1e-12)
    assert O.lse(np.array([[7.5]]), axis=1)[0] == 7.5


def test_plan_argmax_ties_lowest_index():
    S = np.array([[0.1, 0.3, 0.3], [0.2, 0.2, 0.1]])
    assert list(np.argmax(S, axis=1)) == [1, 0]


# ---------------------------------------------------------------- Algorithm 1 end to end

def _small_pair(n=40, seed=31, deg=4.0, anchors=4, d=5, noise=0.0):
    r = rng(seed)
    e1 = erdos_renyi(n, deg, r)
    pi = r.permutation(n)
    e2 = pi[e1]
    X1 = r.standard_normal((n, d))
    X2 = np.zeros_like(X1)
    X2[pi] = X1 + noise * r.standard_normal((n, d))
    pick = r.choice(n, size=anchors, replace=False)
    L = np.stack([pick, pi[pick]], axis=1)
    return e1, e2, X1, X2, L, pi


def _run(n1, e1, n2, e2, X1, X2, L, p, **kw):
    rp1, ci1 = O.build_csr(n1, e1)
    rp2, ci2 = O.build_csr(n2, e2)
    return O.align(n1, rp1, ci1, n2, rp2, ci2, X1, X2, L, p, **kw)


def test_outer_loop_fixed_cost_equals_sinkhorn_at_eps_over_t():
    """lambda_e = lambda_n = 0: t proximal steps from mu nu^T equal one solve at eps/t."""
    n = 12
    e1, e2, X1, X2, L, pi = _small_pair(n=n, seed=32, anchors=2, noise=0.5)
    T = 3
    p = O.Params(eps=0.5, lambda_e=0.0, lambda_n=0.0, lambda_a=0.7, outer_iters=T,
                 inner_iters=20000, tol=1e-14, k_r=3)
    out = _run(n, e1, n, e2, X1, X2, L, p)
    ph = out["phase1"]
    C0 = ph["C_node"] + 0.7 * ph["C_anc"]
    a, b, _, _ = O.sinkhorn(C0, p.eps / T, 40000, tol=1e-14)
    assert np.allclose(out["S"], O.plan(C0, a, b, p.eps / T), atol=1e-11)


@pytest.mark.parametrize("start", ["carry", "mean"])
def test_later_solve_starts_reach_the_same_plans(start):
    """Each inner solve has one optimum whatever its start (up to a constant shift
    of the duals that neither the plan nor the cost update sees): run to convergence,
    starts carried over from the previous solve (or the mean of all earlier solves'
    duals) and zero starts give the same plan at every outer iteration, and the
    non-zero start needs fewer iterations."""
    import dataclasses
    n = 14
    e1, e2, X1, X2, L, pi = _small_pair(n=n, seed=34, anchors=2, noise=0.3)
    # lambda_n = 0 keeps the kernel's dynamic range small enough for every solve to
    # converge to 1e-13 (-log(delta) entries slow Sinkhorn down by orders of magnitude)
    p0 = O.Params(eps=0.3, lambda_n=0.0, outer_iters=3, inner_iters=20000, tol=1e-13, k_r=3)
    zero = _run(n, e1, n, e2, X1, X2, L, p0, keep_history=True)
    carry = _run(n, e1, n, e2, X1, X2, L, dataclasses.replace(p0, dual_start=start), keep_history=True)
    for hz, hc in zip(zero["history"], carry["history"]):
        Sz = O.plan(hz["C"], hz["a"], hz["b"], p0.eps)
        Sc = O.plan(hc["C"], hc["a"], hc["b"], p0.eps)
        assert np.allclose(Sz, Sc, rtol=1e-8, atol=1e-13)
    assert max(zero["errs"] + carry["errs"]) <= 1e-13
    assert carry["iters"][0] == zero["iters"][0]
    assert sum(carry["iters"][1:]) < sum(zero["iters"][1:])


def test_permutation_equivariance():
    n = 30
    e1, e2, X1, X2, L, pi = _small_pair(n=n, seed=33, anchors=3)
    p = O.Params(eps=0.1, outer_iters=3, inner_iters=30)
    base = _run(n, e1, n, e1, X1, X1, np.stack([L[:, 0], L[:, 0]], 1), p)
    perm = _run(n, e1, n, e2, X1, X2, L, p)
    # node j of the self-pair is node pi[j] of the permuted copy
    assert np.allclose(perm["S"][:, pi], base["S"], rtol=1e-10, atol=1e-300)
    assert np.array_equal(pi[base["argmax"]], perm["argmax"])


def test_noise_free_pair_recovers_the_permutation():
    cfg = CONFIGS["er1k"]
    import dataclasses
    cfg0 = dataclasses.replace(cfg, n1=300, noise=0.0, sigma=0.0)
    pr = make_pair(cfg0)
    p = O.Params(eps=cfg.eps, outer_iters=3, inner_iters=30)
    out = _run(pr.n1, pr.edges1, pr.n2, pr.edges2, pr.X1, pr.X2, pr.anchors, p)
    assert (out["argmax"] == pr.truth).mean() == 1.0


def test_four_node_path_vs_path_one_anchor():
    """P4 against itself with one anchor and one-hot features: the identity is recovered
    and the plan is symmetric under the path's reflection only when the anchor is central."""
    e = np.array([[0, 1], [1, 2], [2, 3]])
    X = np.eye(4)
    p = O.Params(eps=0.05, outer_iters=4, inner_iters=300)
    out = _run(4, e, 4, e, X, X, np.array([[0, 0]]), p)
    assert list(out["argmax"]) == [0, 1, 2, 3]
    rows = out["S"].sum(axis=1)
    assert np.allclose(rows, 0.25, atol=1e-12)      # rows are exact after the b-update
    # 4x4 permutation-equivariance under the reflection 0<->3, 1<->2 with anchor (3,3)
    rev = np.array([3, 2, 1, 0])
    out2 = _run(4, e, 4, e, X[rev], X[rev], np.array([[3, 3]]), p)
    assert np.allclose(out2["S"][rev][:, rev], out["S"], rtol=1e-10, atol=0)


# ---------------------------------------------------------------- the pins bite

def test_planted_mistakes_are_caught(monkeypatch):
    """Plant typical slips in the oracle and check a pin above fails for each."""
    C = np.array([[0.3, 0.0], [0.0, 0.0]])
    x = 1.0 / (2.0 * (1.0 + math.exp(0.3 / 0.2)))

    def two_by_two_ok():
        a, b, _, _ = O.sinkhorn(C, 0.1, 2000, tol=1e-15)
        S = O.plan(C, a, b, 0.1)
        return np.allclose(S, [[x, 0.5 - x], [0.5 - x, x]], atol=1e-13)

    assert two_by_two_ok()
    good_plan = O.plan
    # sign slip in the plan exponent
    monkeypatch.setattr(O, "plan", lambda C, a, b, eps: np.exp((a[None, :] + b[:, None] + C) / eps))
    assert not two_by_two_ok()
    monkeypatch.setattr(O, "plan", good_plan)
    # transposed right factor in the neighbourhood product
    n1, n2 = 6, 5
    rp1, ci1 = O.build_csr(n1, tiny_graph(n1, 10, 13))
    rp2, ci2 = O.build_csr(n2, tiny_graph(n2, 9, 14))
    A1, _ = O.row_normalized(n1, rp1, ci1)
    A2, _ = O.row_normalized(n2, rp2, ci2)
    S = rng(17).random((n1, n2))
    M1, M2 = A1.toarray(), A2.toarray()
    P = M1.T @ S @ M2
    wrong = np.asarray((A2 @ (A1.T @ S).T).T)          # uses Abar2^T instead of Abar2
    assert np.allclose(O.nbr_product(A1, A2, S), P) and not np.allclose(wrong, P)


def test_single_entry_forms_match_the_dense_oracle():
    """The per-entry forms used for sampled checks at full size equal the dense steps
    (themselves pinned above) at every sampled (i, j) of a small ragged pair."""
    import dataclasses
    cfg = dataclasses.replace(CONFIGS["er1k"], n1=90, kind="chung_lu", keep_n2=70, anchor_frac=0.1, seed=41)
    pr = make_pair(cfg)
    p = O.Params(eps=0.1, outer_iters=1, inner_iters=5, k_r=4)
    rp1, ci1 = O.build_csr(pr.n1, pr.edges1)
    rp2, ci2 = O.build_csr(pr.n2, pr.edges2)
    ph = O.phase1(pr.n1, rp1, ci1, pr.n2, rp2, ci2, pr.X1, pr.X2, pr.anchors, p)
    X1h, X2h = O.l2_normalize_rows(pr.X1), O.l2_normalize_rows(pr.X2)
    C0 = O.feature_similarity(pr.X1, pr.X2, ph["R1"], ph["R2"], p.alpha)
    Cn = ph["C_node"]
    deg1, deg2 = np.diff(rp1), np.diff(rp2)
    r = rng(42)
    S = r.random((pr.n1, pr.n2)) / (pr.n1 * pr.n2)
    logS = np.log(S) + 0.3
    C = O.cost_update(Cn, ph["C_anc"], ph["C1"], ph["C2"], ph["Abar1"], ph["Abar2"], S, logS, p)
    a, b, _, _ = O.sinkhorn(C, p.eps, 3)
    anchored = set(map(tuple, pr.anchors.tolist()))
    for i, j in zip(r.integers(0, pr.n1, 60), r.integers(0, pr.n2, 60)):
        n1i, n2j = ci1[rp1[i]:rp1[i + 1]], ci2[rp2[j]:rp2[j + 1]]
        assert math.isclose(O.similarity_entry(X1h[i], X2h[j], ph["R1"][i], ph["R2"][j], p.alpha), C0[i, j],
                            rel_tol=1e-12)
        assert math.isclose(O.propagate_entry(C0[np.ix_(n1i, n2j)], deg1[i], deg2[j]), Cn[i, j], rel_tol=1e-12,
                            abs_tol=1e-15)
        c1 = O.intra_row_entries(ph["R1"][i], ph["R1"][n1i], 1.0 / max(deg1[i], 1))
        c2 = O.intra_row_entries(ph["R2"][j], ph["R2"][n2j], 1.0 / deg2[n2j])
        assert np.allclose(c1, ph["C1"][i].toarray()[0, n1i], rtol=1e-12)
        assert np.allclose(c2, ph["C2"][j].toarray()[0, n2j], rtol=1e-12)
        got = O.cost_entry(S[np.ix_(n1i, n2j)], c1, c2, 1.0 / deg1[n1i], 1.0 / deg2[n2j], Cn[i, j],
                           (int(i), int(j)) in anchored, logS[i, j], p)
        assert math.isclose(got, C[i, j], rel_tol=1e-11, abs_tol=1e-11)
        assert math.isclose(O.row_dual_entry(C[i], a, p.eps, pr.n1), b[i], rel_tol=1e-12, abs_tol=1e-13)
        assert math.isclose(O.plan_entry(C[i, j], a[j], b[i], p.eps), O.plan(C, a, b, p.eps)[i, j], rel_tol=1e-12)


def test_true_partner_ranks_vs_rankdata_and_closed_forms():
    """Ranks equal scipy's 'min' ranking of the negated row (1 + number of strictly
    larger scores), ties share the best rank, rows without a partner get 0;
    Hits@K and MRR on hand-made ranks."""
    import scipy.stats as ss
    r = rng(50)
    n1, n2 = 40, 23
    scores = np.round(r.standard_normal((n1, n2)), 1)   # coarse values: ties occur
    truth = r.integers(-3, n2 + 3, n1)
    ranks = O.true_partner_ranks(scores, truth)
    for i in range(n1):
        t = truth[i]
        if 0 <= t < n2:
            assert ranks[i] == ss.rankdata(-scores[i], method="min")[t]
        else:
            assert ranks[i] == 0
    assert (ranks > 0).any() and (ranks == 0).any()
    rk = np.array([1, 2, 0, 10, 1, 4])
    assert O.hits_at_k(rk, 1) == 2 / 5 and O.hits_at_k(rk, 4) == 4 / 5 and O.hits_at_k(rk, 10) == 1.0
    assert math.isclose(O.mean_reciprocal_rank(rk), (1 + 0.5 + 0.1 + 1 + 0.25) / 5)


def test_plan_topk_vs_library_sort_and_stable_brute_force():
    """R16: the top-k lists against numpy's argmax and sort (random plans) and, where
    plan entries tie exactly, against Python's stable sort by explicit loops (equal
    entries keep column order, so the lower column comes first).  Descending order,
    the tie rule and the row/column orientation each break one of these."""
    r = rng(21)
    n1, n2, eps = 7, 23, 0.1
    C, a, b = r.random((n1, n2)), r.normal(size=n2), r.normal(size=n1)
    S = O.plan(C, a, b, eps)
    for k in (1, 5, n2):
        val, idx = O.plan_topk(C, a, b, eps, k)
        assert val.shape == (n1, k) and idx.shape == (n1, k)
        assert np.array_equal(idx[:, 0], np.argmax(S, axis=1))
        np.testing.assert_allclose(val, -np.sort(-S, axis=1)[:, :k], rtol=1e-14)
        np.testing.assert_allclose(val, np.take_along_axis(S, idx, axis=1), rtol=1e-14)
    # k = n2: a permutation of the columns whose values add up to the row sums; after
    # a Sinkhorn b-update the rows carry mu_i = 1/n1 exactly (Eq. (3))
    a2, b2, _, _ = O.sinkhorn(C, eps, 3)
    val, idx = O.plan_topk(C, a2, b2, eps, n2)
    assert all(sorted(row) == list(range(n2)) for row in idx)
    np.testing.assert_allclose(val.sum(axis=1), 1.0 / n1, rtol=1e-12)
    # exact ties: integer costs on a coarse grid, zero duals
    Ct = r.integers(0, 4, size=(n1, n2)).astype(np.float64)
    z2, z1 = np.zeros(n2), np.zeros(n1)
    St = O.plan(Ct, z2, z1, 0.5)
    for k in (3, 9, n2):
        _, idx = O.plan_topk(Ct, z2, z1, 0.5, k)
        for i in range(n1):
            want = sorted(range(n2), key=lambda j: -St[i, j])[:k]   # stable: lower j first on ties
            assert list(idx[i]) == want


@pytest.mark.parametrize("probe", [0, 7])
def test_learned_start_fallback_rule(probe):
    """R17 on the oracle: a learned start whose solve (probe iterations, or the full
    budget with probe 0) misses tol is rerun cold with the full budget; when the cold
    solve ends closer, the run is the cold run itself (plan bit for bit) and both
    solves' iterations count; a start that meets tol is kept with no rerun."""
    import dataclasses
    n = 30
    e1, e2, X1, X2, L, pi = _small_pair(n=n, seed=35, anchors=3, noise=0.3)
    p = O.Params(eps=0.1, outer_iters=2, inner_iters=20, tol=1e-12, warm_probe=probe)
    cold = _run(n, e1, n, e2, X1, X2, L, p)
    bad = np.random.default_rng(3).standard_normal(n) * 50.0          # far from any solution
    with np.errstate(over="ignore"):   # the marginal error of the far start itself overflows
        got = _run(n, e1, n, e2, X1, X2, L, p, b_init=bad)
    budget = probe if probe else p.inner_iters
    assert got["warm_iters"] == budget and got["cold_iters"] == p.inner_iters
    assert got["fell_back"] == 2 and got["warm_err"] > got["cold_err"]
    assert got["iters"][0] == budget + p.inner_iters and got["iters"][1:] == cold["iters"][1:]
    assert np.array_equal(got["S"], cold["S"])
    # a start that meets the tolerance is kept: the converged duals of the first solve
    # (eps 0.3 and lambda_n = 0 keep the kernel's range small enough to converge to 1e-9)
    p2 = dataclasses.replace(p, eps=0.3, tol=1e-9, inner_iters=5000, lambda_n=0.0)
    ref = _run(n, e1, n, e2, X1, X2, L, dataclasses.replace(p2, outer_iters=1))
    good = _run(n, e1, n, e2, X1, X2, L, p2, b_init=ref["b"])
    assert good["fell_back"] == 0 and good["cold_iters"] == -1 and good["warm_err"] <= 1e-9
    assert good["iters"][0] == good["warm_iters"] <= 2


def test_sinkhorn_iterates_obey_the_bounds_behind_the_single_pass():
    """Eq. (3) iterates obey the two bounds that let the single-pass iteration form
    2^y with y = (a_j + b_i - C_ij)/eps in FP32 without a running maximum: after an
    a-update every plan entry is at most nu_j (the column sums are nu_j exactly);
    after a b-update every row sums to mu_i, so the next a-update leaves each row
    sum at least mu_i * min_j nu_j.  The row bound does not hold after the first
    a-update from an arbitrary start, which is why the first two iterations run the
    two-pass form.  Checked on the oracle's own iterates, for costs spread over
    hundreds of eps and for n1 != n2."""
    r = np.random.default_rng(12)
    for n1, n2, eps, spread in [(40, 55, 0.05, 20.0), (70, 30, 0.02, 8.0), (25, 25, 0.1, 50.0)]:
        C = r.random((n1, n2)) * spread + np.add.outer(r.random(n1), r.random(n2)) * spread
        mu, nu = 1.0 / n1, 1.0 / n2
        a = r.standard_normal(n2) * 3.0
        b = r.standard_normal(n1) * 3.0
        b[0] = -200.0 * eps       # a start that starves row 0
        for t in range(12):
            a1, b1, _, _ = O.sinkhorn(C, eps, 1, a0=a, b0=b)
            S_a = O.plan(C, a1, b, eps)     # after the a-update of iteration t
            assert np.allclose(S_a.sum(0), nu, rtol=1e-10, atol=0)
            assert (S_a <= nu * (1 + 1e-10)).all()
            rows = S_a.sum(1)
            if t >= 1:
                assert (rows >= mu * nu * (1 - 1e-10)).all(), (t, rows.min(), mu * nu)
            elif n1 == 40:
                assert rows[0] < 1e-30 * mu * nu    # the starved row: no bound after the first a-update
            S_b = O.plan(C, a1, b1, eps)    # after the b-update
            assert np.allclose(S_b.sum(1), mu, rtol=1e-10, atol=0)
            a, b = a1, b1
