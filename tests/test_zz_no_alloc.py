"""The allocation-free entry point fbsde_solve_noalloc (workspace = the library's fixed device array) against
fbsde_solve with a caller workspace: the same kernels in the same launch shapes, so the outputs agree bit
for bit; two calls in a row, the second with a smaller input; a problem larger than the array is refused.
"""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2510_02635_amd as F  # noqa: E402
from paper_2510_02635_amd import _native as N  # noqa: E402
from paper_2510_02635_amd import workloads  # noqa: E402

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


def _noalloc(pb, x):
    P = x.shape[0]
    u = torch.empty(P, dtype=torch.float64, device=DEV)
    g = torch.empty((P, pb.d), dtype=torch.float64, device=DEV)
    st = torch.empty(P, dtype=torch.int32, device=DEV)
    rc = N.load().fbsde_solve_noalloc(ctypes.byref(pb.c()), P, x.data_ptr(), u.data_ptr(), g.data_ptr(),
                                      st.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, u, g, st


@pytest.mark.parametrize("prec", [F.F64, F.F32C])
def test_noalloc_matches_fbsde_solve_twice(prec):
    cases = [dict(d=300, M=1024, N=4, P=6), dict(d=100, M=512, N=3, P=2)]   # the second call is smaller
    for k, cs in enumerate(cases):
        pb = F.Problem(d=cs["d"], M=cs["M"], N=cs["N"], T=0.3, prec=prec, seed=1, instance=k, **AC)
        x = torch.tensor(workloads.points("normal:0.4", cs["P"], cs["d"], seed=20 + k), device=DEV)
        assert F.workspace_size(pb, cs["P"]) <= F.NOALLOC_SCRATCH_BYTES
        _say(f"[noalloc] call {k}: d={cs['d']} M={cs['M']} N={cs['N']} P={cs['P']} prec={prec}")
        rc, u, g, st = _noalloc(pb, x)
        assert rc == 0
        u1, g1, st1 = F.solve(pb, x)
        torch.cuda.synchronize()
        assert int((st != 0).sum().item()) == 0 and torch.equal(st, st1)
        assert torch.equal(u, u1) and torch.equal(g, g1)


def test_noalloc_refuses_a_problem_beyond_its_array():
    pb = F.Problem(d=1000, M=4096, N=2, T=0.3, prec=F.F32C, **AC)
    P = 8
    assert F.workspace_size(pb, P) > F.NOALLOC_SCRATCH_BYTES
    x = torch.zeros((P, 1000), dtype=torch.float64, device=DEV)
    rc, _, _, _ = _noalloc(pb, x)
    assert rc == N.ENOSPC
