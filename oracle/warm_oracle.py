"""FP64 CPU oracle of the learned warm start (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It mirrors the definitions the library documents for its
warm-start entry points, written independently in numpy:

* per-node inputs of one graph: log(1+deg); log(1 + sum_{k in N(i)} 1/deg_k);
  the 16-dim projection of the L2-normalised attribute row; hop distance to the
  nearest anchor (multi-source BFS, capped at 8) / 8; the random-walk anchor mass
  (Abar^h 1_anchor)_i for h = 1, 2, 3; an is-anchor flag; log(n)/16;
* the fixed Gaussian projection N(0, 1/16): SplitMix64 (Steele, Lea and Flood,
  2014) of the element counter, then the Box-Muller transform;
* a 3-layer MLP  in -> 256 -> 256 -> 1 with SiLU, y = scale * (h2 W3 + b3) + offset,
  its mean-squared-error gradient and one Adam step (Kingma and Ba, 2015).
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np

FEAT, HID, PROJ, HOPS = 24, 256, 16, 8
_M64 = (1 << 64) - 1


def param_count() -> int:
    return FEAT * HID + HID + HID * HID + HID + HID + 1 + 2


def unpack(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + FEAT * HID].reshape(FEAT, HID); o += FEAT * HID
    b1 = p[o:o + HID]; o += HID
    W2 = p[o:o + HID * HID].reshape(HID, HID); o += HID * HID
    b2 = p[o:o + HID]; o += HID
    W3 = p[o:o + HID]; o += HID
    b3 = p[o]; o += 1
    scale, offset = p[o], p[o + 1]
    return W1, b1, W2, b2, W3, b3, scale, offset


def pack(W1, b1, W2, b2, W3, b3, scale, offset) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3, scale, offset]]).astype(np.float64)


# ---------------------------------------------------------------- projection

def splitmix64(z: int) -> int:
    z = (z + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def gauss_projection(d: int, seed: int = 0x5EEDF00D) -> np.ndarray:
    """d x 16 matrix of N(0, 1/16) values: element q uses counters 2q and 2q+1."""
    out = np.empty(d * PROJ)
    for q in range(d * PROJ):
        r1 = splitmix64(seed ^ (2 * q))
        r2 = splitmix64(seed ^ (2 * q + 1))
        u1 = ((r1 >> 11) + 1.0) / 9007199254740992.0
        u2 = (r2 >> 11) / 9007199254740992.0
        out[q] = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2) * 0.25
    return out.reshape(d, PROJ)


# ---------------------------------------------------------------- node inputs

def bfs_hops(n: int, rowptr, colidx, sources, cap: int = HOPS) -> np.ndarray:
    """Multi-source BFS distance, capped at `cap` (unreached nodes get `cap`)."""
    dist = np.full(n, -1, dtype=np.int64)
    q = deque()
    for s in sources:
        if dist[s] < 0:
            dist[s] = 0
            q.append(s)
    while q:
        u = q.popleft()
        if dist[u] >= cap:
            continue
        for e in range(rowptr[u], rowptr[u + 1]):
            v = colidx[e]
            if dist[v] < 0:
                dist[v] = dist[u] + 1
                q.append(v)
    dist[dist < 0] = cap
    return np.minimum(dist, cap)


def node_features(n: int, rowptr, colidx, X, proj, anchor_nodes) -> np.ndarray:
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    deg = np.diff(rowptr).astype(np.float64)
    inv = np.where(deg > 0, 1.0 / np.maximum(deg, 1.0), 0.0)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    F = np.zeros((n, FEAT))
    F[:, 0] = np.log1p(deg)
    sinv = np.zeros(n)
    np.add.at(sinv, rows, inv[colidx])
    F[:, 1] = np.log1p(sinv)
    X = np.asarray(X, dtype=np.float64).reshape(n, -1)
    if X.shape[1] > 0:
        nrm = np.sqrt((X * X).sum(axis=1))
        Xh = np.where(nrm[:, None] > 0, X / np.where(nrm > 0, nrm, 1.0)[:, None], 0.0)
        F[:, 2:2 + PROJ] = Xh @ np.asarray(proj, dtype=np.float64)
    anchor_nodes = np.asarray(anchor_nodes, dtype=np.int64)
    F[:, 18] = bfs_hops(n, rowptr, colidx, anchor_nodes) / HOPS
    r = np.zeros(n)
    r[anchor_nodes] = 1.0
    for h in range(3):
        nxt = np.zeros(n)
        np.add.at(nxt, rows, r[colidx])
        r = nxt * inv
        F[:, 19 + h] = r
    F[anchor_nodes, 22] = 1.0
    F[:, 23] = math.log(n) / 16.0
    return F


# ---------------------------------------------------------------- MLP

def silu(z):
    return z / (1.0 + np.exp(-z))


def mlp_forward(p, x):
    W1, b1, W2, b2, W3, b3, scale, offset = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1 + b1
    h1 = silu(z1)
    z2 = h1 @ W2 + b2
    h2 = silu(z2)
    y = scale * (h2 @ W3 + b3) + offset
    return y, (x, z1, h1, z2, h2)


def mlp_loss_grad(p, x, t):
    """Mean squared error and its gradient with respect to every parameter
    (the scale and offset entries are not trained: zero gradient)."""
    W1, b1, W2, b2, W3, b3, scale, offset = unpack(p)
    y, (x, z1, h1, z2, h2) = mlp_forward(p, x)
    N = x.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(r * r))
    du = 2.0 * r / N * scale                  # d loss / d (h2 W3 + b3)
    gW3 = h2.T @ du
    gb3 = du.sum()
    sig2 = 1.0 / (1.0 + np.exp(-z2))
    dz2 = np.outer(du, W3) * sig2 * (1.0 + z2 * (1.0 - sig2))
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    sig1 = 1.0 / (1.0 + np.exp(-z1))
    dz1 = (dz2 @ W2.T) * sig1 * (1.0 + z1 * (1.0 - sig1))
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3, 0.0, 0.0)


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
