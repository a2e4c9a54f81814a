"""Python front end of libfbsde.so: torch tensors in, torch tensors out.

PyTorch supplies device memory and the current HIP stream; every step of the scheme runs in the
library's HIP kernels.  There is no CPU or PyTorch fallback: a missing library raises.
"""
import ctypes
import math
from dataclasses import dataclass, field
from typing import Optional

import torch

from . import _native as N


@dataclass
class Problem:
    """Problem descriptor (mirrors fbsde_problem).  mu and gvec, when given, are device tensors."""
    d: int
    M: int
    N: int
    T: float
    s: float = math.sqrt(2.0)
    mu: Optional[torch.Tensor] = None
    f_kind: int = N.F_ZERO
    fp: tuple = (0.0, 0.0, 0.0, 0.0)
    g_kind: int = N.G_QUAD
    gp: tuple = (1.0, 0.0, 0.0, 0.0)
    gvec: Optional[torch.Tensor] = None
    eps_h: float = 1.0
    ridge_rel: float = 1e-3
    newton_iters: int = 8
    cg_maxit: int = 500
    cg_rtol: Optional[float] = None        # default: 1e-13 (F64), 1e-7 (F32C)
    cg_fixed_iters: int = 0
    shared_dw: int = 0
    seed: int = 0
    instance: int = 0
    point_base: int = 0
    prec: int = N.F64
    solver: int = N.SOLVER_AUTO             # SOLVER_CG: the matrix-free CG on every level

    def c(self):
        cp = N.CProblem()
        cp.d, cp.M, cp.N, cp.T, cp.s = self.d, self.M, self.N, self.T, self.s
        cp.mu = _ptr(self.mu)
        cp.f_kind, cp.g_kind = self.f_kind, self.g_kind
        cp.fp = (ctypes.c_double * 4)(*[float(v) for v in (list(self.fp) + [0.0] * 4)[:4]])
        cp.gp = (ctypes.c_double * 4)(*[float(v) for v in (list(self.gp) + [0.0] * 4)[:4]])
        cp.gvec = _ptr(self.gvec)
        cp.eps_h, cp.ridge_rel = self.eps_h, self.ridge_rel
        cp.newton_iters, cp.cg_maxit = self.newton_iters, self.cg_maxit
        cp.cg_rtol = self.cg_rtol if self.cg_rtol is not None else (1e-13 if self.prec == N.F64 else 1e-7)
        cp.cg_fixed_iters, cp.shared_dw = self.cg_fixed_iters, self.shared_dw
        cp.seed, cp.instance, cp.point_base = self.seed, self.instance, self.point_base
        cp.prec, cp.solver = self.prec, self.solver
        return cp

    @property
    def state_dtype(self):
        return torch.float64 if self.prec == N.F64 else torch.float32


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors handed to libfbsde must live in device memory")
    return t.data_ptr()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t, shape):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected a contiguous float64 device tensor of shape {tuple(shape)}")
    return t


def state_ld(pb):
    ld = N.load().fbsde_state_ld(ctypes.byref(pb.c()))
    if ld <= 0:
        raise N.FbsdeError("invalid problem descriptor")
    return int(ld)


def workspace_size(pb, P, tape=False):
    out = ctypes.c_size_t(0)
    N.check(N.load().fbsde_workspace_size(ctypes.byref(pb.c()), P, N.WS_TAPE if tape else 0, ctypes.byref(out)))
    return int(out.value)


def workspace(pb, P, tape=False, device="cuda"):
    return torch.empty(max(workspace_size(pb, P, tape), 1), dtype=torch.uint8, device=device)


def terminal(pb, x0):
    """Forward sweep + terminal values: returns (W [P][M][ld], Y [P][M], status [P])."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    ld = state_ld(pb)
    W = torch.empty((P, pb.M, ld), dtype=pb.state_dtype, device=x0.device)
    Y = torch.empty((P, pb.M), dtype=torch.float64, device=x0.device)
    st = torch.empty(P, dtype=torch.int32, device=x0.device)
    N.check(N.load().fbsde_terminal(ctypes.byref(pb.c()), P, x0.data_ptr(), W.data_ptr(), ld, Y.data_ptr(),
                                    st.data_ptr(), _stream()))
    return W, Y, st


def solve_step(pb, k, W, Y_next, x0=None, ws=None):
    """One backward level on caller state W [P][M][ld] (in: W_{k+1}, out: W_k, in place)."""
    P = W.shape[0]
    if W.dtype != pb.state_dtype or not W.is_contiguous() or W.shape[1] != pb.M:
        raise ValueError("state tensor does not match the problem")
    _dev_f64(Y_next, (P, pb.M))
    dev = W.device
    Y = torch.empty((P, pb.M), dtype=torch.float64, device=dev)
    alpha = torch.empty(P, dtype=torch.float64, device=dev)
    alpha_x = torch.empty((P, pb.d), dtype=torch.float64, device=dev)
    st = torch.zeros(P, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(pb, P, device=dev)
    N.check(N.load().fbsde_solve_step(ctypes.byref(pb.c()), P, int(k), _ptr(x0), W.data_ptr(), W.shape[2],
                                      Y_next.data_ptr(), Y.data_ptr(), alpha.data_ptr(), alpha_x.data_ptr(),
                                      st.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return Y, alpha, alpha_x, st


def solve(pb, x0, want_grad=True, tape=False, ws=None, return_iters=False):
    """u(0, x0_p) [P], grad u [P][d] (or None), status [P] (and CG iterations per level)."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    dev = x0.device
    u = torch.empty(P, dtype=torch.float64, device=dev)
    grad = torch.empty((P, pb.d), dtype=torch.float64, device=dev) if want_grad else None
    st = torch.empty(P, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(pb, P, tape=tape, device=dev)
    # the per-level iteration record makes the library wait for each level: only asked for on request
    iters = (ctypes.c_int32 * pb.N)() if return_iters else None
    N.check(N.load().fbsde_solve(ctypes.byref(pb.c()), P, x0.data_ptr(), u.data_ptr(), _ptr(grad), st.data_ptr(),
                                 ws.data_ptr(), ws.numel(), N.WS_TAPE if tape else 0,
                                 ctypes.cast(iters, ctypes.c_void_p) if return_iters else None, _stream()))
    if return_iters:
        return u, grad, st, list(iters)
    return u, grad, st


NOALLOC_SCRATCH_BYTES = 64 << 20


def solve_noalloc(pb, x0, u, grad, status):
    """fbsde_solve_noalloc: the per-point solve with the library's own fixed device scratch array as its
    workspace (no allocation inside the call); u [P], grad [P][d] or None, status [P] are caller tensors."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    _dev_f64(u, (P,))
    if grad is not None:
        _dev_f64(grad, (P, pb.d))
    if status.dtype != torch.int32 or not status.is_cuda or tuple(status.shape) != (P,):
        raise ValueError("status must be an int32 device tensor of shape [P]")
    N.check(N.load().fbsde_solve_noalloc(ctypes.byref(pb.c()), P, x0.data_ptr(), u.data_ptr(), _ptr(grad),
                                         status.data_ptr(), _stream()))
    return u, grad, status


def solve_backward(pb, x0, u_bar, ws, return_iters=False):
    """Adjoint of solve for L = sum_p u_bar[p] u_p; needs ws from solve(..., tape=True).

    Returns x0_bar [P][d], gp_bar [4], fp_bar [4], status [P] (and the adjoint CG iterations per level)."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    _dev_f64(u_bar, (P,))
    dev = x0.device
    x0_bar = torch.empty((P, pb.d), dtype=torch.float64, device=dev)
    gp_bar = torch.zeros(4, dtype=torch.float64, device=dev)
    fp_bar = torch.zeros(4, dtype=torch.float64, device=dev)
    st = torch.zeros(P, dtype=torch.int32, device=dev)
    iters = (ctypes.c_int32 * pb.N)() if return_iters else None
    N.check(N.load().fbsde_solve_backward(ctypes.byref(pb.c()), P, x0.data_ptr(), u_bar.data_ptr(),
                                          x0_bar.data_ptr(), gp_bar.data_ptr(), fp_bar.data_ptr(), st.data_ptr(),
                                          ws.data_ptr(), ws.numel(),
                                          ctypes.cast(iters, ctypes.c_void_p) if return_iters else None, _stream()))
    if return_iters:
        return x0_bar, gp_bar, fp_bar, st, list(iters)
    return x0_bar, gp_bar, fp_bar, st


def normals(pb, p, k, j0, rows, device="cuda"):
    """The increments' normals of rows j0.. of level k (and the raw Philox words)."""
    ng = (pb.d + 3) // 4
    out = torch.empty((rows, pb.d), dtype=torch.float64, device=device)
    words = torch.empty((rows, ng, 4), dtype=torch.int32, device=device)
    N.check(N.load().fbsde_normals(ctypes.byref(pb.c()), p, k, j0, rows, out.data_ptr(), words.data_ptr(),
                                   _stream()))
    return out, words


def box_muller(words, prec):
    """Box-Muller normals [n][4] of Philox words [n][4] (int32 device tensor holding the uint32 bits), as the
    kernels compute them in `prec`."""
    if words.dtype != torch.int32 or not words.is_cuda or not words.is_contiguous() or words.dim() != 2 \
            or words.shape[1] != 4:
        raise ValueError("expected a contiguous int32 device tensor of shape [n][4]")
    out = torch.empty(words.shape, dtype=torch.float64, device=words.device)
    N.check(N.load().fbsde_box_muller(int(prec), words.shape[0], words.data_ptr(), out.data_ptr(), _stream()))
    return out


def launch_timer(on):
    """Start (clearing the record) or stop the library's launch timer of the fused CG product."""
    N.check(N.load().fbsde_launch_timer(1 if on else 0))


TIMED_CG_PRODUCT, TIMED_LITERAL_GRAM, TIMED_LITERAL_ANCHORS, TIMED_CG_LOOP = 0, 1, 2, 3


def workspace_cg_rows(ws):
    """Particle rows streamed by the CG products since the start of the last solve on this workspace
    (its backward pass included); rows x d x element bytes is their algorithmic read traffic."""
    out = ctypes.c_int64(0)
    N.check(N.load().fbsde_workspace_cg_rows(ws.data_ptr(), ctypes.byref(out), _stream()))
    return int(out.value)


def launch_timer_kinds():
    """Kinds (numpy int32, TIMED_*) of the launches recorded by the launch timer, in launch order."""
    import numpy as np
    n = ctypes.c_int64(0)
    N.check(N.load().fbsde_launch_timer_kinds(None, 0, ctypes.byref(n)))
    out = np.zeros(max(n.value, 1), dtype=np.int32)
    N.check(N.load().fbsde_launch_timer_kinds(out.ctypes.data_as(ctypes.c_void_p), out.size, ctypes.byref(n)))
    return out[:n.value]


def launch_timer_read(with_bytes=False):
    """Durations (ms, numpy float32, launch order) of the launches recorded by the launch timer, and with
    `with_bytes` also their algorithmic work (numpy float64: bytes for the CG product, FP64 flops for the
    literal scheme's launches; launch_timer_kinds tells which)."""
    import numpy as np
    n = ctypes.c_int64(0)
    N.check(N.load().fbsde_launch_timer_read(None, None, 0, ctypes.byref(n)))
    out = np.zeros(max(n.value, 1), dtype=np.float32)
    nb = np.zeros(out.size, dtype=np.float64)
    N.check(N.load().fbsde_launch_timer_read(out.ctypes.data_as(ctypes.c_void_p), nb.ctypes.data_as(ctypes.c_void_p),
                                             out.size, ctypes.byref(n)))
    if with_bytes:
        return out[:n.value], nb[:n.value]
    return out[:n.value]


KERNELS = {"cg_matvec": 0, "reverse_newton": 1, "moments": 2, "forward_terminal": 3, "stream_read": 4}


def time_kernel(pb, P, which, ws, reps=5):
    """Average milliseconds of one launch of a hot-path kernel (HIP events on the library's stream)."""
    out = ctypes.c_float(0.0)
    N.check(N.load().fbsde_time_kernel(ctypes.byref(pb.c()), P, KERNELS[which], reps, ws.data_ptr(), ws.numel(),
                                       ctypes.byref(out), _stream()))
    return float(out.value)


class FBSDEFunction(torch.autograd.Function):
    """u(0, x0) as a differentiable function of the points x0 [P][d] and the parameters gp [4], fp [4].

    forward: fbsde_solve with the adjoint tape; backward: fbsde_solve_backward (hand-written reverse mode
    of the whole backward level chain, particles regenerated from their Philox counters).  The gradient
    output grad u is returned as a non-differentiable tensor (second derivatives are not provided).
    """

    @staticmethod
    def forward(ctx, x0, gp, fp, pb):
        from dataclasses import replace
        pbv = replace(pb, gp=tuple(float(v) for v in gp.detach().cpu().tolist()),
                      fp=tuple(float(v) for v in fp.detach().cpu().tolist()))
        P = x0.shape[0]
        ws = workspace(pbv, P, tape=True, device=x0.device)
        u, grad, st = solve(pbv, x0.detach().contiguous(), tape=True, ws=ws)
        ctx.pb, ctx.ws = pbv, ws
        ctx.save_for_backward(x0.detach())
        ctx.gp_meta = (gp.dtype, gp.device)
        ctx.fp_meta = (fp.dtype, fp.device)
        ctx.mark_non_differentiable(grad, st)
        return u, grad, st

    @staticmethod
    def backward(ctx, u_bar, grad_bar, st_bar):
        (x0,) = ctx.saved_tensors
        if u_bar is None:
            u_bar = torch.zeros(x0.shape[0], dtype=torch.float64, device=x0.device)
        x0_bar, gp_bar, fp_bar, _ = solve_backward(ctx.pb, x0, u_bar.to(torch.float64).contiguous(), ctx.ws)
        ctx.ws = None
        return (x0_bar, gp_bar.to(dtype=ctx.gp_meta[0], device=ctx.gp_meta[1]),
                fp_bar.to(dtype=ctx.fp_meta[0], device=ctx.fp_meta[1]), None)


def solve_autograd(pb, x0, gp=None, fp=None):
    """Differentiable solve: returns (u, grad, status); u carries gradients to x0, gp and fp."""
    gp = torch.tensor(pb.gp, dtype=torch.float64) if gp is None else gp
    fp = torch.tensor(pb.fp, dtype=torch.float64) if fp is None else fp
    return FBSDEFunction.apply(x0, gp, fp, pb)


class CoefFBSDEFunction(torch.autograd.Function):
    """u(0, x0) under the affine diagonal coefficients (solve_coef) as a differentiable function of x0, gp
    and fp (the coefficients themselves are constants): forward with the tape, backward through
    fbsde_solve_coef_backward.  grad u and status are non-differentiable outputs."""

    @staticmethod
    def forward(ctx, x0, gp, fp, pb, coef):
        from dataclasses import replace
        pbv = replace(pb, gp=tuple(float(v) for v in gp.detach().cpu().tolist()),
                      fp=tuple(float(v) for v in fp.detach().cpu().tolist()))
        P = x0.shape[0]
        ws = torch.empty(max(coef_workspace_size(pbv, P, *coef, tape=True), 1), dtype=torch.uint8,
                         device=x0.device)
        u, grad, st = solve_coef(pbv, x0.detach().contiguous(), *coef, ws=ws, tape=True)
        ctx.pb, ctx.ws, ctx.coef = pbv, ws, coef
        ctx.save_for_backward(x0.detach())
        ctx.gp_meta = (gp.dtype, gp.device)
        ctx.fp_meta = (fp.dtype, fp.device)
        ctx.mark_non_differentiable(grad, st)
        return u, grad, st

    @staticmethod
    def backward(ctx, u_bar, grad_bar, st_bar):
        (x0,) = ctx.saved_tensors
        if u_bar is None:
            u_bar = torch.zeros(x0.shape[0], dtype=torch.float64, device=x0.device)
        x0_bar, gp_bar, fp_bar, _ = solve_coef_backward(ctx.pb, x0, u_bar.to(torch.float64).contiguous(), ctx.ws,
                                                        *ctx.coef)
        ctx.ws = None
        return (x0_bar, gp_bar.to(dtype=ctx.gp_meta[0], device=ctx.gp_meta[1]),
                fp_bar.to(dtype=ctx.fp_meta[0], device=ctx.fp_meta[1]), None, None)


def solve_coef_autograd(pb, x0, mu0, sigma0, mu1=0.0, sigma1=0.0, gp=None, fp=None):
    """Differentiable solve_coef: returns (u, grad, status); u carries gradients to x0, gp and fp."""
    gp = torch.tensor(pb.gp, dtype=torch.float64) if gp is None else gp
    fp = torch.tensor(pb.fp, dtype=torch.float64) if fp is None else fp
    return CoefFBSDEFunction.apply(x0, gp, fp, pb, (float(mu0), float(sigma0), float(mu1), float(sigma1)))


def gemm(A, B, nt=True, C=None, alpha=1.0, beta=0.0):
    """C = alpha * A op(B) + beta * C on the matrix cores; op(B) = B^T (nt) or B.  float32 / float64."""
    prec = N.F64 if A.dtype == torch.float64 else N.F32C
    m, k = A.shape
    n = B.shape[0] if nt else B.shape[1]
    if C is None:
        C = torch.zeros((m, n), dtype=A.dtype, device=A.device)
    N.check(N.load().fbsde_gemm(prec, 1 if nt else 0, m, n, k, A.data_ptr(), A.stride(0), B.data_ptr(), B.stride(0),
                                C.data_ptr(), C.stride(0), alpha, beta, _stream()))
    return C


def cholesky_solve(K, R=None):
    """In-place blocked Cholesky of K (lower) and in-place solve X K = R of the rows of R; returns info."""
    prec = N.F64 if K.dtype == torch.float64 else N.F32C
    n = K.shape[0]
    P = 0 if R is None else R.shape[0]
    ws = torch.empty(int(N.load().fbsde_cholesky_workspace(prec, n, P)), dtype=torch.uint8, device=K.device)
    info = ctypes.c_int32(0)
    N.check(N.load().fbsde_cholesky_solve(prec, n, K.data_ptr(), K.stride(0), P, None if R is None else R.data_ptr(),
                                          n if R is None else R.stride(0), ws.data_ptr(), ws.numel(),
                                          ctypes.byref(info), _stream()))
    return int(info.value)


def _batch_opts(mode, streams, tile_bytes, max_slots):
    m = {"tiled": N.BATCH_TILED, "persistent": N.BATCH_PERSISTENT}[mode]
    return N.CBatchOpts(m, int(streams), int(tile_bytes), int(max_slots), 0)


def _batch_common(problems, x0s):
    n = len(problems)
    if n != len(x0s) or n == 0:
        raise ValueError("one x0 tensor per problem")
    cps = (N.CProblem * n)(*[pb.c() for pb in problems])
    Ps = (ctypes.c_int64 * n)(*[int(x.shape[0]) for x in x0s])
    for pb, x in zip(problems, x0s):
        _dev_f64(x, (x.shape[0], pb.d))
    return n, cps, Ps


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[None if t is None else t.data_ptr() for t in ts])


def batched_workspace(problems, x0s, adjoint=False, mode="tiled", streams=3, tile_bytes=0, max_slots=512):
    n, cps, Ps = _batch_common(problems, x0s)
    opts = _batch_opts(mode, streams, tile_bytes, max_slots)
    size = ctypes.c_size_t(0)
    N.check(N.load().fbsde_batched_workspace_size(cps, n, ctypes.cast(Ps, ctypes.c_void_p), ctypes.byref(opts),
                                                  1 if adjoint else 0, ctypes.byref(size)))
    return torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=x0s[0].device)


def solve_batched(problems, x0s, want_grad=True, mode="tiled", streams=3, tile_bytes=0, max_slots=512, ws=None):
    """Batched solve of several instances: lists of Problem and of device x0 [P_i][d_i] tensors.

    mode "tiled" (point tiles over `streams` concurrent streams, each tile at most `tile_bytes` of
    workspace, 0 = 8 GiB) or "persistent" (one persistent launch per geometry class, `max_slots`
    workgroups).  Returns lists (u_i, grad_i or None, status_i).
    """
    n, cps, Ps = _batch_common(problems, x0s)
    opts = _batch_opts(mode, streams, tile_bytes, max_slots)
    us, grads, sts = [], [], []
    for pb, x in zip(problems, x0s):
        us.append(torch.empty(x.shape[0], dtype=torch.float64, device=x.device))
        grads.append(torch.empty((x.shape[0], pb.d), dtype=torch.float64, device=x.device) if want_grad else None)
        sts.append(torch.empty(x.shape[0], dtype=torch.int32, device=x.device))
    size = ctypes.c_size_t(0)
    N.check(N.load().fbsde_batched_workspace_size(cps, n, ctypes.cast(Ps, ctypes.c_void_p), ctypes.byref(opts), 0,
                                                  ctypes.byref(size)))
    if ws is None or ws.numel() < size.value:
        ws = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=x0s[0].device)
    gp = _ptrs(grads) if want_grad else None
    N.check(N.load().fbsde_solve_batched(cps, n, ctypes.cast(Ps, ctypes.c_void_p), _ptrs(x0s), _ptrs(us),
                                         None if gp is None else ctypes.cast(gp, ctypes.c_void_p), _ptrs(sts),
                                         ctypes.byref(opts), ws.data_ptr(), ws.numel(), _stream()))
    return us, grads, sts


def batched_cg_bytes(problems, x0s, ws, adjoint=False, streams=3, tile_bytes=0):
    """Algorithmic bytes the CG products of the last tiled batched call on `ws` streamed (same problems, x0
    shapes and options as that call)."""
    n, cps, Ps = _batch_common(problems, x0s)
    opts = _batch_opts("tiled", streams, tile_bytes, 512)
    out = ctypes.c_double(0.0)
    N.check(N.load().fbsde_batched_cg_bytes(cps, n, ctypes.cast(Ps, ctypes.c_void_p), ctypes.byref(opts),
                                            1 if adjoint else 0, ws.data_ptr(), ctypes.byref(out), _stream()))
    return float(out.value)


def solve_batched_backward(problems, x0s, u_bars, streams=3, tile_bytes=0, ws=None):
    """Batched forward + reverse mode: per instance u [P_i], x0_bar [P_i][d_i], gp_bar [4], fp_bar [4], status."""
    n, cps, Ps = _batch_common(problems, x0s)
    opts = _batch_opts("tiled", streams, tile_bytes, 512)
    for ub, x in zip(u_bars, x0s):
        _dev_f64(ub, (x.shape[0],))
    us, xbs, gps, fps, sts = [], [], [], [], []
    for pb, x in zip(problems, x0s):
        us.append(torch.empty(x.shape[0], dtype=torch.float64, device=x.device))
        xbs.append(torch.empty((x.shape[0], pb.d), dtype=torch.float64, device=x.device))
        gps.append(torch.empty(4, dtype=torch.float64, device=x.device))
        fps.append(torch.empty(4, dtype=torch.float64, device=x.device))
        sts.append(torch.empty(x.shape[0], dtype=torch.int32, device=x.device))
    size = ctypes.c_size_t(0)
    N.check(N.load().fbsde_batched_workspace_size(cps, n, ctypes.cast(Ps, ctypes.c_void_p), ctypes.byref(opts), 1,
                                                  ctypes.byref(size)))
    if ws is None or ws.numel() < size.value:
        ws = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=x0s[0].device)
    N.check(N.load().fbsde_solve_batched_backward(cps, n, ctypes.cast(Ps, ctypes.c_void_p), _ptrs(x0s), _ptrs(u_bars),
                                                  _ptrs(us), _ptrs(xbs), _ptrs(gps), _ptrs(fps), _ptrs(sts),
                                                  ctypes.byref(opts), ws.data_ptr(), ws.numel(), _stream()))
    return us, xbs, gps, fps, sts


class CapturedSolve:
    """A solve captured once into a HIP graph (fbsde_graph_capture) and replayed with one launch.

    The graph is bound to this object's tensors: write new points into `x0` in place, call `launch()`,
    read `u`, `grad`, `status`.  Each level's CG solve is one device-side loop, so any descriptor can be
    captured.
    """

    def __init__(self, pb, x0, want_grad=True, tape=False):
        P = x0.shape[0]
        _dev_f64(x0, (P, pb.d))
        dev = x0.device
        self.pb = pb
        self.x0 = x0
        self.u = torch.empty(P, dtype=torch.float64, device=dev)
        self.grad = torch.empty((P, pb.d), dtype=torch.float64, device=dev) if want_grad else None
        self.status = torch.empty(P, dtype=torch.int32, device=dev)
        self.ws = workspace(pb, P, tape=tape, device=dev)
        self._c = pb.c()   # keeps mu / gvec referenced through pb
        h = ctypes.c_void_p()
        N.check(N.load().fbsde_graph_capture(ctypes.byref(self._c), P, x0.data_ptr(), self.u.data_ptr(),
                                             _ptr(self.grad), self.status.data_ptr(), self.ws.data_ptr(),
                                             self.ws.numel(), N.WS_TAPE if tape else 0, ctypes.byref(h), _stream()))
        self._h = h

    def launch(self):
        if self._h is None:
            raise RuntimeError("graph destroyed")
        N.check(N.load().fbsde_graph_launch(self._h, _stream()))
        return self.u, self.grad, self.status

    def close(self):
        if getattr(self, "_h", None) is not None:
            N.check(N.load().fbsde_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CapturedBatch:
    """A tiled batched solve captured once into a HIP graph (fbsde_graph_capture_batched): the fork onto
    the library's stream pool, every tile's level chain and the join back replay with one launch.

    Bound to this object's tensors: write new points into the tensors of `x0s` in place, call
    `launch()`, read `u`, `grad`, `status` (lists per instance)."""

    def __init__(self, problems, x0s, want_grad=True, streams=3, tile_bytes=0):
        n, cps, Ps = _batch_common(problems, x0s)
        self._keep = (cps, Ps)
        opts = _batch_opts("tiled", streams, tile_bytes, 512)
        self.x0s = x0s
        self.u, self.grad, self.status = [], [], []
        for pb, x in zip(problems, x0s):
            self.u.append(torch.empty(x.shape[0], dtype=torch.float64, device=x.device))
            self.grad.append(torch.empty((x.shape[0], pb.d), dtype=torch.float64, device=x.device)
                             if want_grad else None)
            self.status.append(torch.empty(x.shape[0], dtype=torch.int32, device=x.device))
        self.ws = batched_workspace(problems, x0s, streams=streams, tile_bytes=tile_bytes)
        self._ptr_arrays = (_ptrs(x0s), _ptrs(self.u), _ptrs(self.grad) if want_grad else None, _ptrs(self.status))
        xp, up, gp, sp = self._ptr_arrays
        h = ctypes.c_void_p()
        N.check(N.load().fbsde_graph_capture_batched(cps, n, ctypes.cast(Ps, ctypes.c_void_p), xp, up,
                                                     None if gp is None else ctypes.cast(gp, ctypes.c_void_p), sp,
                                                     ctypes.byref(opts), self.ws.data_ptr(), self.ws.numel(),
                                                     ctypes.byref(h), _stream()))
        self._h = h

    def launch(self):
        if self._h is None:
            raise RuntimeError("graph destroyed")
        N.check(N.load().fbsde_graph_launch(self._h, _stream()))
        return self.u, self.grad, self.status

    def close(self):
        if getattr(self, "_h", None) is not None:
            N.check(N.load().fbsde_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(pb, x0, ws=None):
    """Time the candidate launch shapes of the CG product for (precision, d, M, P = len(x0)) and record
    the fastest for every later call with the same key (fbsde_autotune).  Returns the choice as a dict."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    if ws is None:
        ws = workspace(pb, P, device=x0.device)
    r = N.CTuneResult()
    N.check(N.load().fbsde_autotune(ctypes.byref(pb.c()), P, x0.data_ptr(), ws.data_ptr(), ws.numel(),
                                    ctypes.byref(r), _stream()))
    return dict(team=r.team, q=r.q, nchunk=r.nchunk, n_candidates=r.n_candidates, best_ms=r.best_ms,
                default_ms=r.default_ms)


def autotune_reset():
    N.check(N.load().fbsde_autotune_reset())


def literal_workspace_size(pb, P, stored=False):
    """Bytes of workspace for solve_literal; stored=True: the size that keeps every level's particles."""
    out = ctypes.c_size_t(0)
    fn = N.load().fbsde_literal_workspace_size_stored if stored else N.load().fbsde_literal_workspace_size
    N.check(fn(ctypes.byref(pb.c()), P, ctypes.byref(out)))
    return int(out.value)


def _coef(mu0, sigma0, mu1=0.0, sigma1=0.0):
    kind = N.COEF_GEOMETRIC if (mu1 == 0.0 and sigma1 == 0.0) else N.COEF_AFFINE_DIAG
    return N.CCoef(kind, 0, float(mu0), float(sigma0), float(mu1), float(sigma1))


def literal_coef_workspace_size(pb, P, mu0, sigma0, mu1=0.0, sigma1=0.0):
    out = ctypes.c_size_t(0)
    N.check(N.load().fbsde_literal_coef_workspace_size(ctypes.byref(pb.c()), ctypes.byref(_coef(mu0, sigma0, mu1, sigma1)),
                                                       P, ctypes.byref(out)))
    return int(out.value)


def coef_workspace_size(pb, P, mu0, sigma0, mu1=0.0, sigma1=0.0, tape=False):
    out = ctypes.c_size_t(0)
    N.check(N.load().fbsde_coef_workspace_size(ctypes.byref(pb.c()), ctypes.byref(_coef(mu0, sigma0, mu1, sigma1)), P,
                                               N.WS_TAPE if tape else 0, ctypes.byref(out)))
    return int(out.value)


def solve_coef(pb, x0, mu0, sigma0, mu1=0.0, sigma1=0.0, want_grad=True, ws=None, return_iters=False, tape=False):
    """Scheme R (as solve) under the affine diagonal coefficients mu(x) = mu0 x + mu1, sigma(x) =
    diag(sigma0 x + sigma1): u [P], grad [P][d] (or None), status [P] (and CG iterations per level).
    tape=True keeps what solve_coef_backward needs in ws."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    dev = x0.device
    u = torch.empty(P, dtype=torch.float64, device=dev)
    grad = torch.empty((P, pb.d), dtype=torch.float64, device=dev) if want_grad else None
    st = torch.empty(P, dtype=torch.int32, device=dev)
    if ws is None:
        ws = torch.empty(max(coef_workspace_size(pb, P, mu0, sigma0, mu1, sigma1, tape), 1), dtype=torch.uint8,
                         device=dev)
    iters = (ctypes.c_int32 * pb.N)() if return_iters else None
    N.check(N.load().fbsde_solve_coef(ctypes.byref(pb.c()), ctypes.byref(_coef(mu0, sigma0, mu1, sigma1)), P,
                                      x0.data_ptr(), u.data_ptr(), _ptr(grad), st.data_ptr(), ws.data_ptr(),
                                      ws.numel(), N.WS_TAPE if tape else 0,
                                      ctypes.cast(iters, ctypes.c_void_p) if return_iters else None, _stream()))
    if return_iters:
        return u, grad, st, list(iters)
    return u, grad, st


def solve_coef_backward(pb, x0, u_bar, ws, mu0, sigma0, mu1=0.0, sigma1=0.0, return_iters=False):
    """Reverse mode of solve_coef for L = sum_p u_bar[p] u_p; ws from solve_coef(..., tape=True) with the
    same coefficients.  Returns x0_bar [P][d], gp_bar [4], fp_bar [4], status [P] (and the adjoint's CG
    iterations per level)."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    _dev_f64(u_bar, (P,))
    dev = x0.device
    x0_bar = torch.empty((P, pb.d), dtype=torch.float64, device=dev)
    gp_bar = torch.zeros(4, dtype=torch.float64, device=dev)
    fp_bar = torch.zeros(4, dtype=torch.float64, device=dev)
    st = torch.zeros(P, dtype=torch.int32, device=dev)
    iters = (ctypes.c_int32 * pb.N)() if return_iters else None
    N.check(N.load().fbsde_solve_coef_backward(ctypes.byref(pb.c()), ctypes.byref(_coef(mu0, sigma0, mu1, sigma1)), P,
                                               x0.data_ptr(), u_bar.data_ptr(), x0_bar.data_ptr(), gp_bar.data_ptr(),
                                               fp_bar.data_ptr(), st.data_ptr(), ws.data_ptr(), ws.numel(),
                                               ctypes.cast(iters, ctypes.c_void_p) if return_iters else None,
                                               _stream()))
    if return_iters:
        return x0_bar, gp_bar, fp_bar, st, list(iters)
    return x0_bar, gp_bar, fp_bar, st


def sigma_workspace_size(pb, P, tape=False):
    out = ctypes.c_size_t(0)
    N.check(N.load().fbsde_sigma_workspace_size(ctypes.byref(pb.c()), P, N.WS_TAPE if tape else 0, ctypes.byref(out)))
    return int(out.value)


def solve_sigma(pb, x0, sigma, want_grad=True, ws=None, return_iters=False, tape=False):
    """Scheme R (as solve) under the constant diffusion matrix sigma [d][d] (FP64 device tensor):
    u [P], grad [P][d] (or None), status [P] (and CG iterations per level).  tape=True keeps what
    solve_sigma_backward needs in ws."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    _dev_f64(sigma, (pb.d, pb.d))
    dev = x0.device
    u = torch.empty(P, dtype=torch.float64, device=dev)
    grad = torch.empty((P, pb.d), dtype=torch.float64, device=dev) if want_grad else None
    st = torch.empty(P, dtype=torch.int32, device=dev)
    if ws is None:
        ws = torch.empty(max(sigma_workspace_size(pb, P, tape), 1), dtype=torch.uint8, device=dev)
    iters = (ctypes.c_int32 * pb.N)() if return_iters else None
    N.check(N.load().fbsde_solve_sigma(ctypes.byref(pb.c()), sigma.data_ptr(), P, x0.data_ptr(), u.data_ptr(),
                                       _ptr(grad), st.data_ptr(), ws.data_ptr(), ws.numel(),
                                       N.WS_TAPE if tape else 0,
                                       ctypes.cast(iters, ctypes.c_void_p) if return_iters else None, _stream()))
    if return_iters:
        return u, grad, st, list(iters)
    return u, grad, st


def solve_sigma_backward(pb, x0, sigma, u_bar, ws):
    """Reverse mode of solve_sigma for L = sum_p u_bar[p] u_p; ws from solve_sigma(..., tape=True).
    Returns x0_bar [P][d], gp_bar [4], fp_bar [4], status [P]."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    _dev_f64(sigma, (pb.d, pb.d))
    _dev_f64(u_bar, (P,))
    dev = x0.device
    x0_bar = torch.empty((P, pb.d), dtype=torch.float64, device=dev)
    gp_bar = torch.zeros(4, dtype=torch.float64, device=dev)
    fp_bar = torch.zeros(4, dtype=torch.float64, device=dev)
    st = torch.zeros(P, dtype=torch.int32, device=dev)
    N.check(N.load().fbsde_solve_sigma_backward(ctypes.byref(pb.c()), sigma.data_ptr(), P, x0.data_ptr(),
                                                u_bar.data_ptr(), x0_bar.data_ptr(), gp_bar.data_ptr(),
                                                fp_bar.data_ptr(), st.data_ptr(), ws.data_ptr(), ws.numel(), None,
                                                _stream()))
    return x0_bar, gp_bar, fp_bar, st


def solve_literal_geometric(pb, x0, mu0, sigma0, k_stop=0, want_Y=False, want_zstats=False, ws=None, mu1=0.0,
                            sigma1=0.0):
    """Paper-literal per-anchor scheme under the affine diagonal coefficients mu(x) = mu0 x + mu1,
    sigma(x) = diag(sigma0 x + sigma1) (the geometric family when mu1 = sigma1 = 0): outputs as solve_literal."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    dev = x0.device
    u = torch.empty(P, dtype=torch.float64, device=dev)
    st = torch.empty(P, dtype=torch.int32, device=dev)
    Y = torch.empty((P, pb.M), dtype=torch.float64, device=dev) if want_Y else None
    zs = torch.empty((P, pb.M, 2), dtype=torch.float64, device=dev) if want_zstats else None
    if ws is None:
        ws = torch.empty(max(literal_coef_workspace_size(pb, P, mu0, sigma0, mu1, sigma1), 1), dtype=torch.uint8,
                         device=dev)
    N.check(N.load().fbsde_solve_literal_coef(ctypes.byref(pb.c()), ctypes.byref(_coef(mu0, sigma0, mu1, sigma1)), P,
                                              int(k_stop),
                                              x0.data_ptr(), u.data_ptr(), _ptr(Y), _ptr(zs), st.data_ptr(),
                                              ws.data_ptr(), ws.numel(), _stream()))
    return u, st, Y, zs


def solve_literal(pb, x0, k_stop=0, want_Y=False, want_zstats=False, ws=None, stored=False):
    """Paper-literal per-anchor scheme (Algorithm 1 as printed): u [P] = mean_m Y^m_{k_stop}, status [P],
    and optionally Y^m_{k_stop} [P][M] and (|Z^m|^2, sum_i Z^m_i) [P][M][2] at level k_stop.  stored=True
    allocates the workspace that keeps every level's particles (no reversal by regenerated increments)."""
    P = x0.shape[0]
    _dev_f64(x0, (P, pb.d))
    dev = x0.device
    u = torch.empty(P, dtype=torch.float64, device=dev)
    st = torch.empty(P, dtype=torch.int32, device=dev)
    Y = torch.empty((P, pb.M), dtype=torch.float64, device=dev) if want_Y else None
    zs = torch.empty((P, pb.M, 2), dtype=torch.float64, device=dev) if want_zstats else None
    if ws is None:
        ws = torch.empty(max(literal_workspace_size(pb, P, stored), 1), dtype=torch.uint8, device=dev)
    N.check(N.load().fbsde_solve_literal(ctypes.byref(pb.c()), P, int(k_stop), x0.data_ptr(), u.data_ptr(), _ptr(Y),
                                         _ptr(zs), st.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return u, st, Y, zs
