"""The device-side CG loop (one launch per level, fbsde_cgloop.hpp) against the FP64 oracle and against the
host-polled loop it replaced (environment FBSDE_CG_HOST_LOOP=1), over the shapes of its arrival tree:
one chunk per point (no tree), up to eight (one level), and 128 chunks of a single point (three levels).
Also: a solve returns before its work is done (no host wait), a graph captures a solve with the default CG
settings, and the streamed-row record matches the per-level iteration counts.
"""
import os
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2510_02635_amd as F  # noqa: E402
from oracle import scheme as OS  # noqa: E402
from paper_2510_02635_amd import workloads  # noqa: E402

from _convert import problems, rel_err  # noqa: E402

DEV = "cuda"
AC = dict(f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F._native.load()
    F.autotune_reset()


def _host_loop(on):
    if on:
        os.environ["FBSDE_CG_HOST_LOOP"] = "1"
    else:
        os.environ.pop("FBSDE_CG_HOST_LOOP", None)


# (d, M, N, P, prec, tol): nchunk follows from the plan (4096 target blocks over P points, >= 64 rows each)
SHAPES = [
    (30, 100, 3, 5, F.F64, 1e-10),            # one chunk per point: the chunk's block does the CG step
    (100, 512, 4, 3, F.F64, 1e-10),           # eight chunks: one tree level
    (200, 384, 3, 4, F.F64, 1e-10),           # six chunks (a partial fan-in), rank-deficient below d + 1
    (100, 8192, 2, 1, F.F64, 1e-10),          # 128 chunks of one point: three tree levels
    (100, 1024, 3, 4096, F.F64, 1e-10),       # 4096 points of one chunk each, warm-started levels (the
                                              # block's own partials reach its CG step through a barrier)
    (1000, 640, 3, 3, F.F32C, 1e-5),          # FP32C, rank-deficient: FP64 arithmetic in the product
    (64, 2048, 3, 6, F.F32C, 1e-5),           # FP32C, full rank, warm-started
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"d{s[0]}_M{s[1]}_P{s[3]}_{'f64' if s[4] == F.F64 else 'f32c'}"
                                               for s in SHAPES])
def test_device_loop_against_oracle_and_host_loop(shape):
    d, M, N, P, prec, tol = shape
    hp, op = problems(d=d, M=M, N=N, T=0.3, seed=3, instance=2, prec=prec, **AC)
    x0 = workloads.points("normal:0.4", P, d, seed=d + M)
    xt = torch.tensor(x0, device=DEV)
    _say(f"[cgloop] d={d} M={M} N={N} P={P} prec={prec}")
    _host_loop(False)
    u, g, st, it = F.solve(hp, xt, return_iters=True)
    torch.cuda.synchronize()
    _host_loop(True)
    try:
        uh, gh, sth, ith = F.solve(hp, xt, return_iters=True)
        torch.cuda.synchronize()
    finally:
        _host_loop(False)
    _say(f"  iterations per level: device {it} host {ith}")
    assert int((st != 0).sum().item()) == 0 and int((sth != 0).sum().item()) == 0
    # the two loops differ only in the order the chunk partials are summed (more than four chunks), which
    # can move a level's stopping test by one iteration
    assert all(abs(a - b) <= 1 for a, b in zip(it, ith))
    assert rel_err(u.cpu().numpy(), uh.cpu().numpy()) <= (1e-13 if prec == F.F64 else 1e-6)
    assert rel_err(g.cpu().numpy(), gh.cpu().numpy()) <= (1e-11 if prec == F.F64 else 1e-5)
    for p in sorted({0, P - 1}):
        ref = OS.solve_point(op, x0[p], p)
        eu = abs(u[p].item() - ref["u"]) / abs(ref["u"])
        eg = rel_err(g[p].cpu().numpy(), ref["grad"])
        _say(f"  p={p} rel_u={eu:.2e} rel_grad={eg:.2e}")
        assert eu <= tol and eg <= tol


def test_device_loop_adjoint_against_host_loop():
    d, M, N, P = 80, 600, 3, 4
    hp, op = problems(d=d, M=M, N=N, T=0.3, seed=5, instance=1, **AC)
    x0 = workloads.points("normal:0.3", P, d, seed=9)
    xt = torch.tensor(x0, device=DEV)
    ub = torch.ones(P, dtype=torch.float64, device=DEV)
    out = []
    for host in (False, True):
        _host_loop(host)
        try:
            ws = F.workspace(hp, P, tape=True)
            F.solve(hp, xt, tape=True, ws=ws)
            xb, gpb, fpb, st, it = F.solve_backward(hp, xt, ub, ws, return_iters=True)
            torch.cuda.synchronize()
            out.append((xb.cpu().numpy(), gpb.cpu().numpy(), st.cpu().numpy(), it))
        finally:
            _host_loop(False)
    assert all(abs(a - b) <= 1 for a, b in zip(out[0][3], out[1][3]))
    assert rel_err(out[0][0], out[1][0]) <= 1e-12 and rel_err(out[0][1], out[1][1]) <= 1e-12
    assert not out[0][2].any()
    ref = OS.adjoint_point(op, x0[1], 1, ubar=1.0)
    assert rel_err(out[0][0][1], ref["x0bar"]) <= 1e-10


def test_streamed_rows_match_iteration_counts():
    # one point: the largest iteration count of a level is the point's own, so the rows streamed by all
    # products of the solve are M x (sum over levels of the iterations)
    d, M, N = 50, 700, 4
    hp, _ = problems(d=d, M=M, N=N, T=0.3, seed=1, instance=0, **AC)
    xt = torch.tensor(workloads.points("normal:0.5", 1, d, seed=2), device=DEV)
    ws = F.workspace(hp, 1)
    _, _, st, it = F.solve(hp, xt, ws=ws, return_iters=True)
    rows = F.workspace_cg_rows(ws)
    _say(f"[cgloop] rows {rows} iterations {it}")
    assert int(st.item()) == 0
    assert rows == M * sum(it)


def test_solve_returns_before_its_work_is_done():
    # d = 1000, 256 points, M = 4096, N = 10 in FP32C: about a tenth of a second of GPU work, enqueued in
    # a few milliseconds of host time
    d, M, N, P = 1000, 4096, 10, 256
    hp, _ = problems(d=d, M=M, N=N, T=0.3, seed=0, instance=1, prec=F.F32C, **AC)
    xt = torch.tensor(workloads.points("normal:0.5", P, d, seed=1), device=DEV)
    ws = F.workspace(hp, P)
    F.solve(hp, xt, ws=ws)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, g, st = F.solve(hp, xt, ws=ws)
    t1 = time.perf_counter()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _say(f"[cgloop] host call {1e3 * (t1 - t0):.2f} ms, until done {1e3 * (t2 - t0):.2f} ms")
    assert int((st != 0).sum().item()) == 0
    assert (t1 - t0) < 0.25 * (t2 - t0)


def test_graph_capture_with_default_cg_settings():
    d, M, N, P = 100, 512, 5, 2
    hp, op = problems(d=d, M=M, N=N, T=0.3, seed=0, instance=0, **AC)
    x0 = workloads.points("normal:0.3", P, d, seed=4)
    xt = torch.tensor(x0, device=DEV)
    u0, g0, _ = F.solve(hp, xt)
    torch.cuda.synchronize()
    cs = F.CapturedSolve(hp, xt)
    for rep in range(3):
        u, g, st = cs.launch()
        torch.cuda.synchronize()
        assert torch.equal(u, u0) and torch.equal(g, g0) and int((st != 0).sum().item()) == 0
        torch.zeros(1024, device=DEV).sum().item()   # eager work between replays
    ref = OS.solve_point(op, x0[0], 0)
    assert abs(u0[0].item() - ref["u"]) <= 1e-10 * abs(ref["u"])


@pytest.mark.parametrize("fam", ["ac", "hj"])
def test_many_points_few_chunks_no_wait_limit(fam):
    # 64 points of 6 chunks each (d = 500, M = 100, FP64): two points per work queue, twelve items per
    # queue and as many blocks.  With queues that reused their slots every lap, a block that held a ticket
    # and completed a stolen item's point could wait for its own ticket's slot until the wait bound (the
    # level then took 2 s and its points were flagged).  The HJ-type case also has right-hand sides of
    # 1e-150 to 1e-180 at the late levels (its terminal value is a d = 500 Gaussian), whose squared norms
    # leave the normal range unless the CG solves for a power-of-two-scaled right-hand side: without the
    # scaling one level ran to the iteration cap and the points went non-finite.  Every level must end at
    # once with every point converged and equal to the oracle.
    d, M, N, T, P = 500, 100, 10, 0.5, 64
    if fam == "hj":
        kw = dict(f_kind=F.F_HJ_SINK, fp=(0.1, 0, 0, 0), g_kind=F.G_HJ_GAUSS, gp=(0.5, 0, 0, 0))
    else:
        kw = dict(AC)
    # the CG on every level (this cloud would otherwise take the direct dual solve)
    hp, op = problems(d=d, M=M, N=N, T=T, seed=0, instance=9, solver=F.SOLVER_CG, **kw)
    x0 = np.zeros((P, d)) if fam == "hj" else workloads.points("normal:0.05", P, d, seed=3)
    xt = torch.tensor(x0, device=DEV)
    ws = F.workspace(hp, P)
    _say(f"[cgloop many points] f={fam} d={d} M={M} N={N} P={P}")
    F.solve(hp, xt, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, g, st, it = F.solve(hp, xt, ws=ws, return_iters=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    _say(f"  {sec * 1e3:.1f} ms, iterations per level {it}")
    assert not st.cpu().numpy().any()
    assert max(it) < hp.cg_maxit
    assert sec < 1.0
    u, g = u.cpu().numpy(), g.cpu().numpy()
    for p in (0, 17, 63):
        ref = OS.solve_point(op, x0[p], p)
        assert abs(u[p] - ref["u"]) <= 1e-10 * abs(ref["u"])
        assert rel_err(g[p], ref["grad"]) <= 1e-10
