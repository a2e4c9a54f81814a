"""GPU parity of the persistent batched launch (fbsde_solve_batched) against the FP64 oracle.

Instances of uneven d (several geometry classes, team widths 1..16 waves), M, f, g and precision run in
one call with fewer workgroup slots than points, so slots are reused through the work queue.  Each
instance must equal the oracle at the precision bar (FP64 1e-10, FP32C 1e-5).
"""
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


INSTANCES = [
    (dict(d=37, M=100, N=3, T=0.5, f_kind=F.F_HJB, fp=(0.8, 0, 0, 0), g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0), seed=7,
          instance=0), "uniform", 5),
    (dict(d=37, M=150, N=3, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
          instance=1), "normal:0.3", 3),
    (dict(d=600, M=130, N=2, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
          instance=2), "normal:0.2", 2),
    (dict(d=1500, M=70, N=2, T=0.3, f_kind=F.F_ZERO, g_kind=F.G_QUAD, prec=F.F32C, instance=3), "normal:0.5", 2),
    (dict(d=3000, M=64, N=2, T=1.0, f_kind=F.F_HJB, fp=(1.3, 0, 0, 0), g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0),
          instance=4), "uniform", 1),
    (dict(d=200, M=400, N=4, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
          instance=5), "normal_over_sqrt_d", 3),   # M > d + 1: warm-started CG
]


@pytest.mark.parametrize("max_slots", [3, 64])
def test_batched_matches_oracle(max_slots):
    hps, ops, xs = [], [], []
    for kw, xkind, P in INSTANCES:
        hp, op = problems(**kw)
        hps.append(hp)
        ops.append(op)
        xs.append(workloads.points(xkind, P, kw["d"], 21 + kw["instance"]))
    _say(f"[batched] {len(hps)} instances, max_slots={max_slots}")
    us, gs, sts = F.solve_batched(hps, [torch.tensor(x, device=DEV) for x in xs], max_slots=max_slots)
    torch.cuda.synchronize()
    for i, (hp, op, x) in enumerate(zip(hps, ops, xs)):
        tol = 1e-10 if hp.prec == F.F64 else 1e-5
        u, g, st = us[i].cpu().numpy(), gs[i].cpu().numpy(), sts[i].cpu().numpy()
        for p in range(x.shape[0]):
            ref = OS.solve_point(op, x[p], p)
            eu = abs(u[p] - ref["u"]) / abs(ref["u"])
            eg = rel_err(g[p], ref["grad"])
            _say(f"  inst {i} d={hp.d} M={hp.M} p={p} rel_u={eu:.2e} rel_grad={eg:.2e}")
            assert st[p] == 0
            assert eu <= tol and eg <= tol


def test_batched_equals_single_solve():
    kw, xkind, P = INSTANCES[5]
    hp, _ = problems(**kw)
    x = torch.tensor(workloads.points(xkind, P, kw["d"], 99), device=DEV)
    us, gs, _ = F.solve_batched([hp], [x], max_slots=2)
    u1, g1, _ = F.solve(hp, x)
    torch.cuda.synchronize()
    assert torch.allclose(us[0], u1, rtol=1e-12, atol=0)
    assert torch.allclose(gs[0], g1, rtol=1e-10, atol=1e-14)
