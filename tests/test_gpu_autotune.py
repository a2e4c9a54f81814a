"""GPU: the autotuner's recorded launch shape is used by later solves, which stay at the parity bar.

fbsde_autotune times the fused CG product over the row split (team width) and the per-point chunk
split; the solve with the recorded shape must match the FP64 oracle like the default one (only the
summation order of the partial sums changes), and the workspace never grows."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2510_02635_amd as F  # noqa: E402
from oracle import scheme as OS  # noqa: E402
from paper_2510_02635_amd import workloads  # noqa: E402

from _convert import problems, rel_err  # noqa: E402

DEV = "cuda"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F._native.load()
    yield
    F.autotune_reset()


@pytest.mark.parametrize("prec,tol", [(F.F64, 1e-10), (F.F32C, 1e-5)], ids=["fp64", "fp32c"])
def test_tuned_shape_keeps_parity(prec, tol):
    kw = dict(d=1200, M=700, N=3, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0))
    hp, op = problems(prec=prec, **kw)
    P = 6
    x0 = workloads.points("normal_over_sqrt_d", P, kw["d"], 4)
    xt = torch.tensor(x0, device=DEV)
    F.autotune_reset()
    w0 = F.workspace_size(hp, P)
    u0, g0, _ = F.solve(hp, xt)
    res = F.autotune(hp, xt)
    _say(f"[autotune] {prec}: {res}")
    assert res["n_candidates"] >= 2 and res["best_ms"] <= res["default_ms"] * 1.0001
    assert F.workspace_size(hp, P) <= w0
    u, g, st = F.solve(hp, xt)
    torch.cuda.synchronize()
    assert int(st.abs().sum().item()) == 0
    for p in range(P):
        ref = OS.solve_point(op, x0[p], p)
        eu = abs(u[p].item() - ref["u"]) / abs(ref["u"])
        eg = rel_err(g[p].cpu().numpy(), ref["grad"])
        _say(f"  p={p} rel_u={eu:.2e} rel_grad={eg:.2e}")
        assert eu <= tol and eg <= tol
    F.autotune_reset()
    u1, g1, _ = F.solve(hp, xt)
    torch.cuda.synchronize()
    assert torch.equal(u1, u0) and torch.equal(g1, g0)   # the default shape again, bit for bit


@pytest.mark.parametrize("prec", [F.F64, F.F32C], ids=["fp64", "fp32c"])
def test_kernel_timer_and_read_ceiling(prec):
    # every timed kernel returns a positive duration; the read-ceiling stream leaves the state bytes as they were
    hp, _ = problems(d=300, M=256, N=2, T=0.3, prec=prec, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                     gp=(0.4, 0, 0, 0))
    P = 5
    xt = torch.tensor(workloads.points("normal:0.3", P, 300, 2), device=DEV)
    ws = F.workspace(hp, P)
    F.solve(hp, xt, ws=ws)
    torch.cuda.synchronize()
    state_bytes = P * hp.M * F.state_ld(hp) * (8 if prec == F.F64 else 4)
    before = ws[:state_bytes].clone()
    ms = F.time_kernel(hp, P, "stream_read", ws, reps=3)
    _say(f"[timer] {prec}: stream_read {ms:.4f} ms")
    assert ms > 0 and torch.equal(ws[:state_bytes], before)
    for which in ("cg_matvec", "reverse_newton", "moments", "forward_terminal"):
        t = F.time_kernel(hp, P, which, ws, reps=2)
        _say(f"  {which} {t:.4f} ms")
        assert t > 0


def test_launch_timer_records_every_cg_product(monkeypatch):
    hp, _ = problems(d=300, M=256, N=3, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                     gp=(0.4, 0, 0, 0), solver=F.SOLVER_CG)
    xt = torch.tensor(workloads.points("normal:0.3", 4, 300, 2), device=DEV)
    ws = F.workspace(hp, 4)
    F.solve(hp, xt, ws=ws)
    torch.cuda.synchronize()
    # the device-side loop: one timed launch per level, whose work is the rows its products streamed
    F.launch_timer(True)
    _, _, st, iters = F.solve(hp, xt, ws=ws, return_iters=True)
    F.launch_timer(False)
    ms, nb = F.launch_timer_read(with_bytes=True)
    rows = F.workspace_cg_rows(ws)
    _say(f"[launch timer] {ms.size} loop launches for per-level iterations {iters}, mean {ms.mean():.4f} ms, "
         f"{rows} rows streamed")
    assert ms.size == 3 and np.all(F.launch_timer_kinds() == F.TIMED_CG_LOOP) and np.all(nb == 0)
    assert 256 * sum(iters) <= rows <= 4 * 256 * sum(iters)
    assert np.all(ms > 0) and int(st.abs().sum().item()) == 0
    # the host-polled loop: one record per product
    monkeypatch.setenv("FBSDE_CG_HOST_LOOP", "1")
    F.launch_timer(True)
    _, _, st, iters = F.solve(hp, xt, ws=ws, return_iters=True)
    F.launch_timer(False)
    monkeypatch.delenv("FBSDE_CG_HOST_LOOP")
    ms, nb = F.launch_timer_read(with_bytes=True)
    _say(f"[launch timer] {ms.size} product launches for per-level iterations {iters}, mean {ms.mean():.4f} ms")
    assert np.all(nb == 4 * 256 * 300 * 8)   # points x particles x d x FP64 bytes
    # the host loop polls every 8 iterations, so each level launches at most 7 more products than it needs
    assert sum(iters) <= ms.size <= sum(iters) + 7 * len(iters)
    assert np.all(ms > 0) and int(st.abs().sum().item()) == 0
    # stopped: a further solve adds nothing; restarting clears the record
    F.solve(hp, xt, ws=ws)
    assert F.launch_timer_read().size == ms.size
    F.launch_timer(True)
    F.launch_timer(False)
    assert F.launch_timer_read().size == 0
