"""Pins of the warm-start oracle: finite differences, closed forms, library special cases."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

from oracle import fastalign_oracle as O
from oracle import warm_oracle as W


def small_params(seed=0, scale=1.0, offset=0.0):
    r = np.random.default_rng(seed)
    W1 = r.standard_normal((W.FEAT, W.HID)) / math.sqrt(W.FEAT)
    b1 = r.standard_normal(W.HID) * 0.1
    W2 = r.standard_normal((W.HID, W.HID)) / math.sqrt(W.HID)
    b2 = r.standard_normal(W.HID) * 0.1
    W3 = r.standard_normal(W.HID) / math.sqrt(W.HID)
    return W.pack(W1, b1, W2, b2, W3, 0.3, scale, offset)


def test_param_count_matches_layout():
    assert W.param_count() == 24 * 256 + 256 + 256 * 256 + 256 + 256 + 3
    p = small_params()
    assert p.size == W.param_count()
    assert all(np.shares_memory(u, p) or np.ndim(u) == 0 for u in W.unpack(p)[:5])


def test_mlp_gradient_matches_central_differences():
    r = np.random.default_rng(1)
    p = small_params(2, scale=1.7, offset=0.4)
    x = r.standard_normal((7, W.FEAT))
    t = r.standard_normal(7)
    loss, g = W.mlp_loss_grad(p, x, t)
    offs = [0, W.FEAT * W.HID, W.FEAT * W.HID + W.HID, W.FEAT * W.HID + 2 * W.HID + W.HID * W.HID,
            W.param_count() - 3 - W.HID]
    idx = set(r.integers(0, W.param_count() - 3, size=40).tolist()) | {o + 3 for o in offs} | {W.param_count() - 3}
    h = 1e-6
    for i in sorted(idx):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (W.mlp_loss_grad(pp, x, t)[0] - W.mlp_loss_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert g[-2] == 0.0 and g[-1] == 0.0


def test_mlp_forward_linear_regime():
    """With large positive pre-activations SiLU is the identity to 1e-30: the network
    reduces to the affine map scale*(((x W1 + b1) W2 + b2) W3 + b3) + offset."""
    r = np.random.default_rng(3)
    W1 = np.abs(r.standard_normal((W.FEAT, W.HID)))
    b1 = np.full(W.HID, 100.0)
    W2 = np.abs(r.standard_normal((W.HID, W.HID))) * 0.01
    b2 = np.full(W.HID, 100.0)
    W3 = r.standard_normal(W.HID)
    p = W.pack(W1, b1, W2, b2, W3, 0.5, 2.0, -1.0)
    x = np.abs(r.standard_normal((5, W.FEAT)))
    y, _ = W.mlp_forward(p, x)
    lin = 2.0 * ((((x @ W1) + b1) @ W2 + b2) @ W3 + 0.5) - 1.0
    assert np.allclose(y, lin, rtol=1e-12)


def test_adam_first_step_closed_form():
    r = np.random.default_rng(4)
    p, g = r.standard_normal(50), r.standard_normal(50)
    p1, m, v = W.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-8)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_splitmix64_reference_sequence():
    # first three outputs of SplitMix64 from state 0 (Steele, Lea, Flood 2014)
    z = 0
    outs = []
    for _ in range(3):
        outs.append(W.splitmix64(z))
        z = (z + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_gauss_projection_statistics():
    P = W.gauss_projection(256)
    assert P.shape == (256, 16)
    assert abs(P.mean()) < 0.02 and abs(P.std() - 0.25) < 0.01


def test_bfs_hops_vs_shortest_paths():
    r = np.random.default_rng(5)
    n = 60
    e = r.integers(0, n, size=(70, 2))
    rp, ci = O.build_csr(n, e)
    A = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(n, n))
    src = np.array([3, 17, 40])
    D = csg.shortest_path(A, unweighted=True, indices=src).min(axis=0)
    want = np.where(np.isfinite(D), np.minimum(D, 8), 8)
    assert np.array_equal(W.bfs_hops(n, rp, ci, src), want.astype(np.int64))


def test_node_features_walk_mass_and_degrees():
    r = np.random.default_rng(6)
    n, d = 40, 5
    e = r.integers(0, n, size=(60, 2))
    rp, ci = O.build_csr(n, e)
    X = r.standard_normal((n, d))
    proj = r.standard_normal((d, 16))
    nodes = np.array([1, 7, 22])
    F = W.node_features(n, rp, ci, X, proj, nodes)
    Abar, deg = O.row_normalized(n, rp, ci)
    M = Abar.toarray()
    one = np.zeros(n)
    one[nodes] = 1
    for h in range(1, 4):
        assert np.allclose(F[:, 18 + h], np.linalg.matrix_power(M, h) @ one, atol=1e-15)
    assert np.allclose(F[:, 0], np.log1p(deg))
    sinv = np.array([sum(1.0 / deg[k] for k in ci[rp[i]:rp[i + 1]]) for i in range(n)])
    assert np.allclose(F[:, 1], np.log1p(sinv))
    Xh = X / np.linalg.norm(X, axis=1, keepdims=True)
    assert np.allclose(F[:, 2:18], Xh @ proj)
    assert set(np.nonzero(F[:, 22])[0]) == set(nodes) and np.allclose(F[:, 23], math.log(n) / 16)
