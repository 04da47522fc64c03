"""Writes the stored expected values under tests/golden/.

The paper prints no worked example with numbers (its evaluation reports timings
and accuracy on datasets), so the fixtures come from two sources:

* sinkhorn_2x2.json: the closed form of the 2 x 2 problem with uniform marginals
  (Eq. (1) solved by Eq. (3)/(4)): for C = [[delta, 0], [0, 0]] the optimal plan is
  [[x, 1/2 - x], [1/2 - x, x]] with x = 1 / (2 (1 + exp(delta / (2 eps)))).  Written
  from the formula, not from the oracle.
* align_small_oracle.json: inputs and outputs of Algorithm 1 on two tiny pairs as
  computed by the FP64 oracle (this script calls nothing but oracle/), kept as a
  regression reference for the oracle and as stored expected values for the GPU.

Usage (repository root): python tests/golden/make_golden.py
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import fastalign_oracle as O  # noqa: E402


def two_by_two():
    cases = []
    for delta, eps in [(1.0, 0.5), (0.3, 0.1), (-2.0, 0.25), (0.05, 0.02)]:
        x = 1.0 / (2.0 * (1.0 + math.exp(delta / (2.0 * eps))))
        cases.append(dict(C=[[delta, 0.0], [0.0, 0.0]], eps=eps, plan=[[x, 0.5 - x], [0.5 - x, x]]))
    return dict(source="closed form of the 2x2 uniform-marginal problem (Eq. (1), Eq. (3), Eq. (4))", cases=cases)


def align_case(name, n1, e1, n2, e2, X1, X2, anchors, params):
    rp1, ci1 = O.build_csr(n1, np.asarray(e1, dtype=np.int64).reshape(-1, 2))
    rp2, ci2 = O.build_csr(n2, np.asarray(e2, dtype=np.int64).reshape(-1, 2))
    p = O.Params(**params)
    out = O.align(n1, rp1, ci1, n2, rp2, ci2, np.asarray(X1, float), np.asarray(X2, float),
                  np.asarray(anchors, dtype=np.int64).reshape(-1, 2), p)
    return dict(name=name, n1=n1, n2=n2, edges1=np.asarray(e1).tolist(), edges2=np.asarray(e2).tolist(),
                X1=np.asarray(X1).tolist(), X2=np.asarray(X2).tolist(), anchors=np.asarray(anchors).tolist(),
                params=params, S=out["S"].tolist(), a=out["a"].tolist(), b=out["b"].tolist(),
                argmax=[int(v) for v in out["argmax"]], errs=[float(v) for v in out["errs"]],
                iters=[int(v) for v in out["iters"]])


def small_alignments():
    cases = []
    path = [[0, 1], [1, 2], [2, 3]]
    cases.append(align_case("P4 vs P4, one anchor, one-hot attributes", 4, path, 4, path, np.eye(4), np.eye(4),
                            [[0, 0]], dict(eps=0.05, outer_iters=4, inner_iters=100)))
    r = np.random.default_rng(2607)
    n = 12
    e1 = np.stack([r.integers(0, n, 30), r.integers(0, n, 30)], 1)
    perm = r.permutation(n)
    e2 = perm[e1]
    X1 = r.standard_normal((n, 3))
    X2 = np.empty_like(X1)
    X2[perm] = X1 + 0.1 * r.standard_normal((n, 3))
    anchors = np.stack([np.arange(3), perm[:3]], 1)
    cases.append(align_case("12-node random pair, relabelled copy, 3 anchors", n, e1, n, e2, X1, X2, anchors,
                            dict(eps=0.1, outer_iters=3, inner_iters=60)))
    return dict(source="FP64 oracle (Algorithm 1), written by tests/golden/make_golden.py", cases=cases)


if __name__ == "__main__":
    with open(os.path.join(HERE, "sinkhorn_2x2.json"), "w") as f:
        json.dump(two_by_two(), f, indent=1)
    with open(os.path.join(HERE, "align_small_oracle.json"), "w") as f:
        json.dump(small_alignments(), f)
    print("wrote", os.listdir(HERE))
