"""GPU: a solve captured into a HIP graph (fbsde_graph_capture) replays exactly the eager launch sequence.

Each replay follows eager work of the program itself (new points written into the bound x0, a torch
reduction, a synchronisation) and must equal the eager fbsde_solve on the same points bit for bit; the
per-point form runs with a fixed number of CG launches (each exits at once for a converged point), which
must give the same values as the polled solve."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2510_02635_amd as F  # noqa: E402
from paper_2510_02635_amd import workloads  # noqa: E402

DEV = "cuda"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F._native.load()


CASES = [
    ("c0_fp64", dict(d=100, M=512, N=5, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                     gp=(0.4, 0, 0, 0), cg_fixed_iters=96), 3),
    ("fp32c_rank_deficient", dict(d=700, M=96, N=3, T=0.3, f_kind=F.F_HJB, fp=(0.8, 0, 0, 0), g_kind=F.G_HJB_LOG,
                                  gp=(1.0, 0, 0, 0), prec=F.F32C, cg_fixed_iters=96), 4),
    ("shared_fp32c", dict(d=300, M=200, N=3, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                          gp=(0.4, 0, 0, 0), prec=F.F32C, shared_dw=1), 33),
    # a small rank-deficient cloud: the direct dual solve on every level, captured
    ("fp64_dual", dict(d=200, M=64, N=3, T=0.3, f_kind=F.F_HJB, fp=(0.8, 0, 0, 0), g_kind=F.G_HJB_LOG,
                       gp=(1.0, 0, 0, 0)), 3),
]


@pytest.mark.parametrize("name,kw,P", CASES, ids=[c[0] for c in CASES])
def test_graph_replays_equal_eager(name, kw, P):
    pb = F.Problem(**kw)
    x0 = torch.tensor(workloads.points("normal:0.3", P, kw["d"], 1), device=DEV)
    _say(f"[graph] {name}: capture")
    g = F.CapturedSolve(pb, x0)
    for rep in range(3):
        new = torch.tensor(workloads.points("normal:0.3", P, kw["d"], 10 + rep), device=DEV)
        g.x0.copy_(new)
        _ = (new * new).sum().item()          # eager work and a synchronisation between replays
        u, gr, st = g.launch()
        torch.cuda.synchronize()
        ue, ge, ste = F.solve(pb, new.clone())
        torch.cuda.synchronize()
        _say(f"  replay {rep}: |du|={float((u - ue).abs().max()):.2e} |dgrad|={float((gr - ge).abs().max()):.2e}")
        assert torch.equal(u, ue) and torch.equal(gr, ge) and torch.equal(st, ste)
        assert int(st.abs().sum().item()) == 0
        if kw.get("cg_fixed_iters"):
            # the converging CG (stopping per point) gives the bits of the fixed launch count
            kw_poll = dict(kw, cg_fixed_iters=0, solver=F.SOLVER_CG)
            up, gp_, _ = F.solve(F.Problem(**kw_poll), new.clone())
            torch.cuda.synchronize()
            assert torch.equal(u, up) and torch.equal(gr, gp_)
    g.close()


def test_graph_flags_points_short_of_the_fixed_launches():
    kw = dict(d=100, M=512, N=2, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
              cg_fixed_iters=2)
    pb = F.Problem(**kw)
    x0 = torch.tensor(workloads.points("normal:0.3", 2, 100, 2), device=DEV)
    _say("[graph] too few CG launches")
    g = F.CapturedSolve(pb, x0)
    _, _, st = g.launch()
    torch.cuda.synchronize()
    assert np.all((st.cpu().numpy() & 1) == 1)   # FBSDE_ST_CG_MAXIT
    g.close()
