"""Host-side properties of every workspace-size entry point over many shapes (no GPU: sizing only plans).

Run as part of the CPU suite, and against the host-sanitized library by `python -m paper_2510_02635_amd.hostsan
tests/test_host_sizes.py`: randomized descriptors drive the planning, carving and tile-plan code of the host side.

* A tape never shrinks a workspace, and a workspace holds at least the state (P x M x row pitch).
* The x-dependent coefficient form needs at least the per-point workspace (its tables come after it); its taped
  FP32C size equals the FP64 one exactly for rank-deficient designs (M <= d + 1), whose reverse mode keeps an FP64
  state.
* The batched tiled plan is at least the largest single tile's arena.
"""
import ctypes

import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import paper_2510_02635_amd as F  # noqa: E402
from paper_2510_02635_amd import _native as N  # noqa: E402

SHAPES = st.tuples(st.integers(1, 3000), st.integers(2, 3000), st.integers(1, 40), st.integers(1, 300),
                   st.sampled_from([F.F64, F.F32C]), st.sampled_from([F.F_ALLEN_CAHN, F.F_HJB, F.F_BURGERS]))


def _pb(d, M, N_, prec, fk):
    return F.Problem(d=d, M=M, N=N_, T=0.3, prec=prec, f_kind=fk, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC,
                     gp=(0.4, 0, 0, 0))


@settings(max_examples=60, deadline=None, derandomize=True)
@given(SHAPES)
def test_per_point_sizes(shape):
    d, M, N_, P, prec, fk = shape
    pb = _pb(d, M, N_, prec, fk)
    a = F.workspace_size(pb, P)
    b = F.workspace_size(pb, P, tape=True)
    # the state itself is a lower bound (the chunking, and with it the partial sums, depends on P, so the
    # size need not grow monotonically with P)
    state = P * M * F.state_ld(pb) * (8 if prec == F.F64 else 4)
    assert state <= a <= b
    assert a % 256 == 0 and b % 256 == 0


@settings(max_examples=60, deadline=None, derandomize=True)
@given(SHAPES, st.sampled_from([(0.1, 0.3, 0.0, 0.0), (-0.8, 0.0, 0.2, 0.5), (0.05, 0.2, -0.1, 0.4)]))
def test_coef_sizes(shape, coef):
    d, M, N_, P, prec, fk = shape
    pb = _pb(d, M, N_, prec, fk)
    a = F.coef_workspace_size(pb, P, *coef)
    b = F.coef_workspace_size(pb, P, *coef, tape=True)
    assert F.workspace_size(pb, P) <= a <= b
    if prec == F.F32C:
        b64 = F.coef_workspace_size(_pb(d, M, N_, F.F64, fk), P, *coef, tape=True)
        assert (b == b64) == (M <= d + 1)


@settings(max_examples=40, deadline=None, derandomize=True)
@given(st.lists(st.tuples(st.integers(1, 2000), st.integers(2, 2000), st.integers(0, 64)), min_size=1, max_size=6),
       st.integers(1, 8))
def test_batched_plan_covers_every_tile(insts, streams):
    pbs = [_pb(d, M, 3, F.F32C, F.F_HJB) for d, M, _ in insts]
    Ps = [P for _, _, P in insts]
    o = N.CBatchOpts(N.BATCH_TILED, streams, 0, 0, 0)
    cps = (N.CProblem * len(pbs))(*[pb.c() for pb in pbs])
    Pa = (ctypes.c_int64 * len(Ps))(*Ps)
    out = ctypes.c_size_t(0)
    rc = N.load().fbsde_batched_workspace_size(cps, len(pbs), ctypes.cast(Pa, ctypes.c_void_p), ctypes.byref(o), 0,
                                               ctypes.byref(out))
    assert rc == N.OK
    for pb, P in zip(pbs, Ps):
        if P > 0:
            assert out.value >= F.workspace_size(pb, 1)
