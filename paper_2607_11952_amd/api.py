"""Python front end of the HIP library: device memory from PyTorch, calls through the C ABI.

PyTorch only allocates device buffers and supplies the current HIP stream;
every computation happens in libfastalign.so.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import binding as B


def _lib():
    return B.load()


def _ptr(t: Optional[torch.Tensor]):
    """Raw device address of a dense row-major tensor (the ABI has no strides)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("fastalign: tensors passed to the C ABI must be contiguous (row-major)")
    return t.data_ptr() if t.numel() > 0 else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(device=None):
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


# ------------------------------------------------------------------ graphs

def csr_build(n: int, edges: np.ndarray):
    """Host CSR of an undirected edge list through fa_csr_build (bit-exact, sorted rows)."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).reshape(-1, 2))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    nnz = C.c_int64(0)
    cap = 2 * e.shape[0]
    colidx = np.zeros(max(cap, 1), dtype=np.int32)
    _lib().call("fa_csr_build", n, e.shape[0], e.ctypes.data if e.size else None, rowptr.ctypes.data,
                colidx.ctypes.data, cap, C.byref(nnz))
    return rowptr, colidx[: nnz.value].copy()


@dataclasses.dataclass
class DeviceCSR:
    n: int
    rowptr: torch.Tensor   # int64 [n+1]
    colidx: torch.Tensor   # int32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.colidx.numel())

    @property
    def c(self) -> B.fa_csr:
        s = B.fa_csr()
        s.n, s.nnz = self.n, self.nnz
        s.rowptr = _ptr(self.rowptr)
        s.colidx = _ptr(self.colidx)
        return s

    @staticmethod
    def from_host(n: int, rowptr: np.ndarray, colidx: np.ndarray, device=None) -> "DeviceCSR":
        d = _dev(device)
        return DeviceCSR(n, torch.from_numpy(np.asarray(rowptr, np.int64)).to(d),
                         torch.from_numpy(np.asarray(colidx, np.int32)).to(d))

    @staticmethod
    def from_edges(n: int, edges: np.ndarray, device=None) -> "DeviceCSR":
        rp, ci = csr_build(n, edges)
        return DeviceCSR.from_host(n, rp, ci, device)


# ------------------------------------------------------------------ parameters

def params(**kw) -> B.fa_params:
    """fa_params with the library defaults; lambda_p and eps_anchor follow eps unless given."""
    p = _lib().default_params()
    for k, v in kw.items():
        if k in ("plan_dtype", "feat_dtype") and isinstance(v, str):
            v = {"f32": B.FA_F32, "bf16": B.FA_BF16}[v]
        if k == "dual_start" and isinstance(v, str):
            v = {"zero": B.FA_START_ZERO, "carry": B.FA_START_CARRY, "mean": B.FA_START_MEAN}[v]
        if k in ("feat_l2norm", "warm_start", "profile", "dual_start", "transpose_cost", "plan_in_ct",
                 "warm_fallback", "warm_probe", "sink_fused"):
            v = int(v)
        setattr(p, k, v)
    if p.plan_in_ct and "transpose_cost" not in kw:
        p.transpose_cost = 1  # the working plan lives in the C^T buffer
    if "lambda_p" not in kw:
        p.lambda_p = p.eps
    if "eps_anchor" not in kw:
        p.eps_anchor = p.eps
    return p


def _sdt(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return B.FA_F32
    if t.dtype == torch.bfloat16:
        return B.FA_BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


# ------------------------------------------------------------------ Phase 1

def row_normalize(A: DeviceCSR) -> torch.Tensor:
    inv = torch.empty(A.n, dtype=torch.float32, device=A.rowptr.device)
    _lib().call("fa_row_normalize", C.byref(A.c), _ptr(inv), _stream())
    return inv


def positional(A: DeviceCSR, inv: torch.Tensor, nodes: torch.Tensor, beta: float, k: int) -> torch.Tensor:
    nL = int(nodes.numel())
    R = torch.empty((A.n, nL), dtype=torch.float32, device=inv.device)
    Rt = torch.empty_like(R)
    _lib().call("fa_positional", C.byref(A.c), _ptr(inv), _ptr(nodes), nL, float(beta), int(k), _ptr(R),
                _ptr(Rt), _stream())
    return R


def sddmm(A: DeviceCSR, inv: torch.Tensor, R: torch.Tensor, by_col: bool) -> torch.Tensor:
    out = torch.empty(A.nnz, dtype=torch.float32, device=inv.device)
    _lib().call("fa_sddmm", C.byref(A.c), _ptr(inv), _ptr(R), int(R.shape[1]), int(by_col), _ptr(out), _stream())
    return out


def l2_normalize(X: torch.Tensor, dtype=torch.float32) -> torch.Tensor:
    out = torch.empty(X.shape, dtype=dtype, device=X.device)
    _lib().call("fa_l2_normalize", _ptr(X), X.shape[0], X.shape[1], _ptr(out), _sdt(out), _stream())
    return out


def feature_sim(X1, X2, R1, R2, alpha: float) -> torch.Tensor:
    n1, n2 = X1.shape[0], X2.shape[0]
    d, nL = X1.shape[1], R1.shape[1]
    out = torch.empty((n1, n2), dtype=torch.float32, device=X1.device)
    _lib().call("fa_feature_sim", _ptr(X1), _ptr(X2), n1, n2, d, _sdt(X1), _ptr(R1), _ptr(R2), nL, _sdt(R1),
                float(alpha), _ptr(out), _stream())
    return out


def propagate(A1: DeviceCSR, inv1, A2: DeviceCSR, inv2, C_in: torch.Tensor, k: int, chunk_rows: int = 0):
    Cm = C_in.clone()
    tmp = torch.empty_like(Cm)
    nb = _lib().raw("fa_cost_workspace_size")(A1.n, A2.n, B.FA_F32, chunk_rows)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=Cm.device)
    _lib().call("fa_propagate", C.byref(A1.c), _ptr(inv1), C.byref(A2.c), _ptr(inv2), _ptr(Cm), _ptr(tmp), int(k),
                int(chunk_rows), _ptr(ws), nb, _stream())
    return Cm


# ------------------------------------------------------------------ Phase 2 / 3

def cost(A1, A2, w1, w2, inv1, inv2, S, C_node, partner, a, b, p: B.fa_params, C_prev: torch.Tensor,
         transposed: bool = False):
    """The rebuilt cost (a new tensor); with transposed=True also C^T: returns (C, Ct)."""
    Cm = C_prev.clone()
    Ct = torch.empty((C_prev.shape[1], C_prev.shape[0]), dtype=torch.float32, device=Cm.device) if transposed else None
    nb = _lib().raw("fa_cost_workspace_size")(A1.n, A2.n, _sdt(S), p.chunk_rows)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=Cm.device)
    _lib().call("fa_cost", C.byref(A1.c), C.byref(A2.c), _ptr(w1), _ptr(w2), _ptr(inv1), _ptr(inv2), _ptr(S),
                _sdt(S), _ptr(C_node), _ptr(partner), _ptr(a), _ptr(b), C.byref(p), _ptr(Cm), _ptr(Ct), _ptr(ws), nb,
                _stream())
    return (Cm, Ct) if transposed else Cm


def sinkhorn(Cm: torch.Tensor, eps: float, a: torch.Tensor, b: torch.Tensor, max_iter: int, tol: float = 0.0,
             check_every: int = 1, Ct: Optional[torch.Tensor] = None):
    """Runs in place on a, b (FP64); returns (iterations, marginal error).  Ct (C^T,
    contiguous n2 x n1) selects the transposed column pass."""
    n1, n2 = Cm.shape
    nb = _lib().raw("fa_sinkhorn_workspace_size")(n1, n2)
    ws = torch.empty(nb, dtype=torch.uint8, device=Cm.device)
    di = torch.zeros(1, dtype=torch.int32, device=Cm.device)
    de = torch.zeros(1, dtype=torch.float64, device=Cm.device)
    hi, he = C.c_int32(0), C.c_double(0)
    _lib().call("fa_sinkhorn", _ptr(Cm), _ptr(Ct), n1, n2, float(eps), _ptr(a), _ptr(b), int(max_iter), float(tol),
                int(check_every), _ptr(di), _ptr(de), C.byref(hi), C.byref(he), _ptr(ws), nb, _stream())
    return hi.value, he.value


def sinkhorn_fused(Cm: torch.Tensor, eps: float, a: torch.Tensor, b: torch.Tensor, max_iter: int, tol: float = 0.0,
                   check_every: int = 1):
    """The single-pass iteration (one read of C per iteration); in place on a, b.
    Returns (iterations, marginal error)."""
    n1, n2 = Cm.shape
    nb = _lib().raw("fa_sinkhorn_fused_workspace_size")(n1, n2)
    ws = torch.empty(nb, dtype=torch.uint8, device=Cm.device)
    di = torch.zeros(1, dtype=torch.int32, device=Cm.device)
    de = torch.zeros(1, dtype=torch.float64, device=Cm.device)
    hi, he = C.c_int32(0), C.c_double(0)
    _lib().call("fa_sinkhorn_fused", _ptr(Cm), n1, n2, float(eps), _ptr(a), _ptr(b), int(max_iter), float(tol),
                int(check_every), _ptr(di), _ptr(de), C.byref(hi), C.byref(he), _ptr(ws), nb, _stream())
    return hi.value, he.value


def sinkhorn_fused_grid(n1: int, n2: int):
    """(row groups, partners per row) of the single pass on the current device, or None."""
    gr, gc = C.c_int32(0), C.c_int32(0)
    st = _lib().raw("fa_sinkhorn_fused_grid")(int(n1), int(n2), C.byref(gr), C.byref(gc))
    return (gr.value, gc.value) if st == 0 else None


def plan(Cm: torch.Tensor, eps: float, a: torch.Tensor, b: torch.Tensor, dtype=torch.float32, argmax: bool = False,
         truth: Optional[torch.Tensor] = None):
    """S (and argmax if asked; and the true partners' ranks if truth is given)."""
    n1, n2 = Cm.shape
    S = torch.empty((n1, n2), dtype=dtype, device=Cm.device)
    am = torch.empty(n1, dtype=torch.int32, device=Cm.device) if argmax else None
    rk = torch.empty(n1, dtype=torch.int32, device=Cm.device) if truth is not None else None
    _lib().call("fa_plan", _ptr(Cm), n1, n2, float(eps), _ptr(a), _ptr(b), _ptr(S), _sdt(S), _ptr(am), _ptr(truth),
                _ptr(rk), _stream())
    out = (S,) + ((am,) if argmax else ()) + ((rk,) if truth is not None else ())
    return out if len(out) > 1 else S


def plan_topk(Cm: torch.Tensor, eps: float, a: torch.Tensor, b: torch.Tensor, k: int):
    """Per-row top-k of the plan without writing it: (values float32 [n1, k], columns int32 [n1, k])."""
    n1, n2 = Cm.shape
    val = torch.empty((n1, k), dtype=torch.float32, device=Cm.device)
    idx = torch.empty((n1, k), dtype=torch.int32, device=Cm.device)
    _lib().call("fa_plan_topk", _ptr(Cm), n1, n2, float(eps), _ptr(a), _ptr(b), int(k), _ptr(val), _ptr(idx),
                _stream())
    return val, idx


# ------------------------------------------------------------------ end to end

@dataclasses.dataclass
class AlignInputs:
    A1: DeviceCSR
    A2: DeviceCSR
    X1: torch.Tensor
    X2: torch.Tensor
    anchors: torch.Tensor   # int32 [nL, 2]

    @staticmethod
    def from_pair(pair, device=None) -> "AlignInputs":
        d = _dev(device)
        return AlignInputs(DeviceCSR.from_edges(pair.n1, pair.edges1, d), DeviceCSR.from_edges(pair.n2, pair.edges2, d),
                           torch.from_numpy(np.ascontiguousarray(pair.X1, np.float32)).to(d),
                           torch.from_numpy(np.ascontiguousarray(pair.X2, np.float32)).to(d),
                           torch.from_numpy(np.ascontiguousarray(pair.anchors, np.int32)).to(d))


@dataclasses.dataclass
class AlignResult:
    S: Optional[torch.Tensor]   # None when the run kept no dense plan (plan_in_ct without one)
    a: torch.Tensor
    b: torch.Tensor
    argmax: torch.Tensor
    stats: B.fa_stats
    status: int
    rank: Optional[torch.Tensor] = None   # rank of each row's true partner (0: none), if asked for
    topk_val: Optional[torch.Tensor] = None   # final plan's per-row top-k, if asked for
    topk_idx: Optional[torch.Tensor] = None


def workspace_bytes(inp: AlignInputs, p: B.fa_params) -> int:
    return int(_lib().raw("fa_align_workspace_size")(inp.A1.n, inp.A2.n, int(inp.X1.shape[1]),
                                                     int(inp.anchors.shape[0]), inp.A1.nnz, inp.A2.nnz, C.byref(p)))


class Aligner:
    """Holds the workspace and outputs for repeated fa_align calls on one input."""

    def __init__(self, inp: AlignInputs, p: B.fa_params, mlp: Optional[torch.Tensor] = None,
                 truth: Optional[torch.Tensor] = None, topk: int = 0, dense_plan: bool = True):
        """truth (int32[n1] on the device, -1 = no partner) makes run() also rank each
        row's true partner in the final plan (AlignResult.rank); topk > 0 returns the
        final plan's per-row top-k lists; dense_plan = False (needs p.plan_in_ct)
        allocates no n1 x n2 plan at all."""
        if not dense_plan and not p.plan_in_ct:
            raise ValueError("dense_plan=False needs plan_in_ct=1")
        self.inp, self.p, self.mlp, self.truth, self.topk = inp, p, mlp, truth, int(topk)
        n1, n2 = inp.A1.n, inp.A2.n
        dev = inp.X1.device
        self.ws_bytes = workspace_bytes(inp, p)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        sd = torch.bfloat16 if p.plan_dtype == B.FA_BF16 else torch.float32
        self.S = torch.empty((n1, n2), dtype=sd, device=dev) if dense_plan else None
        self.a = torch.empty(n2, dtype=torch.float64, device=dev)
        self.b = torch.empty(n1, dtype=torch.float64, device=dev)
        self.argmax = torch.empty(n1, dtype=torch.int32, device=dev)
        self.rank = torch.empty(n1, dtype=torch.int32, device=dev) if truth is not None else None
        self.topk_val = torch.empty((n1, self.topk), dtype=torch.float32, device=dev) if self.topk else None
        self.topk_idx = torch.empty((n1, self.topk), dtype=torch.int32, device=dev) if self.topk else None

    # ---- one outer iteration at a time (fa_align_begin / fa_align_step / fa_align_end)
    def _common(self):
        inp = self.inp
        return (C.byref(inp.A1.c), C.byref(inp.A2.c), int(inp.X1.shape[1]), int(inp.anchors.shape[0]),
                C.byref(self.p))

    def begin(self, acc: Optional[B.fa_stats] = None):
        """Phase 1 and S^0 (synchronises for the anchor check and at the end); acc receives
        its device time (phase_ms[0]) and, with p.profile, its kernels' timings."""
        inp = self.inp
        _lib().call("fa_align_begin", C.byref(inp.A1.c), C.byref(inp.A2.c), _ptr(inp.X1), _ptr(inp.X2),
                    int(inp.X1.shape[1]), _ptr(inp.anchors), int(inp.anchors.shape[0]), C.byref(self.p),
                    _ptr(self.S), _ptr(self.a), _ptr(self.b), C.byref(acc) if acc is not None else None,
                    _ptr(self.ws), self.ws_bytes, _stream())

    def step(self, t: int, last: bool = False, acc: Optional[B.fa_stats] = None):
        """Outer iteration t; with last=True its plan pass also writes argmax (and ranks)."""
        A1, A2, d, nL, p = self._common()
        _lib().call("fa_align_step", A1, A2, d, nL, p, _ptr(self.mlp), int(t), _ptr(self.S), _ptr(self.a),
                    _ptr(self.b), _ptr(self.argmax) if last else None, _ptr(self.truth) if last else None,
                    _ptr(self.rank) if last else None, C.byref(acc) if acc is not None else None, _ptr(self.ws),
                    self.ws_bytes, _stream())

    def end(self, steps: int, stats: Optional[B.fa_stats] = None) -> AlignResult:
        A1, A2, d, nL, p = self._common()
        st = stats if stats is not None else B.fa_stats()
        status = _lib().call("fa_align_end", A1, A2, d, nL, p, int(steps), _ptr(self.S), _ptr(self.a), _ptr(self.b),
                             _ptr(self.argmax) if steps == 0 else None, _ptr(self.truth) if steps == 0 else None,
                             _ptr(self.rank) if steps == 0 else None, self.topk, _ptr(self.topk_val),
                             _ptr(self.topk_idx), C.byref(st), _ptr(self.ws), self.ws_bytes, _stream())
        return AlignResult(self.S, self.a, self.b, self.argmax, st, status, self.rank, self.topk_val, self.topk_idx)

    def run(self) -> AlignResult:
        st = B.fa_stats()
        inp = self.inp
        status = _lib().call("fa_align", C.byref(inp.A1.c), C.byref(inp.A2.c), _ptr(inp.X1), _ptr(inp.X2),
                             int(inp.X1.shape[1]), _ptr(inp.anchors), int(inp.anchors.shape[0]), C.byref(self.p),
                             _ptr(self.mlp), _ptr(self.S), _ptr(self.a), _ptr(self.b), _ptr(self.argmax),
                             _ptr(self.truth), _ptr(self.rank), self.topk, _ptr(self.topk_val), _ptr(self.topk_idx),
                             C.byref(st), _ptr(self.ws), self.ws_bytes, _stream())
        return AlignResult(self.S, self.a, self.b, self.argmax, st, status, self.rank, self.topk_val, self.topk_idx)


def align(inp: AlignInputs, p: B.fa_params, mlp: Optional[torch.Tensor] = None,
          truth: Optional[torch.Tensor] = None, topk: int = 0, dense_plan: bool = True) -> AlignResult:
    return Aligner(inp, p, mlp, truth, topk, dense_plan).run()


# ------------------------------------------------------------------ warm start pieces

def node_features(A: DeviceCSR, inv: torch.Tensor, X: torch.Tensor, nodes: torch.Tensor,
                  proj: Optional[torch.Tensor] = None) -> torch.Tensor:
    F = int(_lib().raw("fa_node_feature_dim")())
    out = torch.empty((A.n, F), dtype=torch.float32, device=inv.device)
    nb = _lib().raw("fa_node_features_workspace_size")(A.n)
    ws = torch.empty(nb, dtype=torch.uint8, device=inv.device)
    _lib().call("fa_node_features", C.byref(A.c), _ptr(inv), _ptr(X), int(X.shape[1]), _ptr(proj), _ptr(nodes),
                int(nodes.numel()), _ptr(out), _ptr(ws), nb, _stream())
    return out


def mlp_param_count() -> int:
    return int(_lib().raw("fa_mlp_param_count")())


def mlp_act(N: int, device) -> torch.Tensor:
    return torch.empty(int(_lib().raw("fa_mlp_act_floats")(N)), dtype=torch.float32, device=device)


def mlp_forward(prm: torch.Tensor, x: torch.Tensor, act: Optional[torch.Tensor] = None):
    N = x.shape[0]
    act = mlp_act(N, x.device) if act is None else act
    y = torch.empty(N, dtype=torch.float32, device=x.device)
    _lib().call("fa_mlp_forward", _ptr(prm), _ptr(x), N, _ptr(y), _ptr(act), _stream())
    return y, act


def mlp_backward(prm: torch.Tensor, x: torch.Tensor, t: torch.Tensor, act: torch.Tensor):
    grad = torch.empty_like(prm)
    loss = torch.zeros(1, dtype=torch.float64, device=x.device)
    _lib().call("fa_mlp_backward", _ptr(prm), _ptr(x), _ptr(t), x.shape[0], _ptr(act), _ptr(grad), _ptr(loss),
                _stream())
    return grad, loss


def adam_step(prm, grad, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _lib().call("fa_adam_step", _ptr(prm), _ptr(grad), _ptr(m), _ptr(v), prm.numel(), float(lr), float(beta1),
                float(beta2), float(eps), int(step), _stream())


def stream_read(x, partial, nblocks: int):
    """One streaming read of x (float32, numel a multiple of 4) on the current stream."""
    _lib().call("fa_stream_read", _ptr(x), x.numel(), _ptr(partial), int(nblocks), _stream())
