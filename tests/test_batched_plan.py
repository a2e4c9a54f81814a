"""Host-side checks of the batched scheduler's tile plan (no GPU: fbsde_batched_workspace_size only plans).

Tiled schedule: each instance is cut into equal point tiles, each the largest whose single-instance
workspace fits the tile cap (at least one point); the workspace is a [tiles][8] FP64 header with eight
64-bit per-stream traffic counters after it, plus one arena (the largest tile workspace) per stream,
streams = min(requested, tiles)."""
import ctypes

import pytest

import paper_2510_02635_amd as F
from paper_2510_02635_amd import _native as N


def _size(pbs, Ps, adjoint=0, **opts):
    o = N.CBatchOpts(opts.get("mode", N.BATCH_TILED), opts.get("streams", 0), opts.get("tile_bytes", 0),
                     opts.get("max_slots", 0), opts.get("reserved", 0))
    cps = (N.CProblem * len(pbs))(*[pb.c() for pb in pbs])
    P = (ctypes.c_int64 * len(Ps))(*Ps)
    out = ctypes.c_size_t(0)
    rc = N.load().fbsde_batched_workspace_size(cps, len(pbs), ctypes.cast(P, ctypes.c_void_p), ctypes.byref(o),
                                               adjoint, ctypes.byref(out))
    return rc, int(out.value)


def _round(x, a=256):
    return (x + a - 1) // a * a


def _expected(pbs, Ps, tile_bytes, streams, tape=False):
    tiles, arena = 0, 0
    for pb, P in zip(pbs, Ps):
        if P == 0:
            continue
        np_ = 1
        for m in range(min(P, 65535), 0, -1):
            if F.workspace_size(pb, m, tape) <= tile_bytes:
                np_ = m
                break
        nt = -(-P // np_)
        np_ = -(-P // nt)
        for p0 in range(0, P, np_):
            arena = max(arena, _round(F.workspace_size(pb, min(np_, P - p0), tape)))
            tiles += 1
    nw = min(streams, max(tiles, 1))
    return _round(tiles * 64 + 64) + nw * arena


PBS = [F.Problem(d=37, M=100, N=3, T=0.5), F.Problem(d=600, M=130, N=2, T=0.3),
       F.Problem(d=1500, M=70, N=2, T=0.3, prec=N.F32C), F.Problem(d=200, M=400, N=4, T=0.3)]
PS = [5, 3, 0, 7]


@pytest.mark.parametrize("tile_bytes,streams", [(1 << 20, 3), (1 << 24, 4), (1 << 33, 2), (1, 8)])
def test_tiled_workspace_follows_the_tile_plan(tile_bytes, streams):
    rc, got = _size(PBS, PS, tile_bytes=tile_bytes, streams=streams)
    assert rc == 0
    assert got == _expected(PBS, PS, tile_bytes, streams)


def test_tiled_adjoint_workspace_uses_the_tape():
    rc0, a = _size(PBS, PS, tile_bytes=1 << 22, streams=2)
    rc1, b = _size(PBS, PS, adjoint=1, tile_bytes=1 << 22, streams=2)
    assert rc0 == 0 and rc1 == 0 and b == _expected(PBS, PS, 1 << 22, 2, tape=True) and b > a


@pytest.mark.parametrize("opts", [dict(streams=9), dict(streams=-1), dict(mode=2), dict(tile_bytes=-5),
                                  dict(reserved=1), dict(max_slots=-3)])
def test_bad_options_rejected(opts):
    assert _size(PBS, PS, **opts)[0] == N.EINVAL


def test_persistent_has_no_adjoint_and_no_shared_form():
    assert _size(PBS, PS, adjoint=1, mode=N.BATCH_PERSISTENT)[0] == N.EINVAL
    shared = F.Problem(d=40, M=64, N=2, T=0.3, shared_dw=1)
    assert _size([shared], [4], mode=N.BATCH_PERSISTENT)[0] == N.EINVAL
    assert _size([shared], [4])[0] == 0                      # tiled forward: allowed
    assert _size([shared], [4], adjoint=1)[0] == 0             # tiled forward + reverse mode: allowed


def test_points_beyond_one_launch_are_tiled():
    # one launch carries at most 65535 points (grid.y); the tiled schedule cuts larger instances
    pb = F.Problem(d=4, M=64, N=2, T=0.3)
    rc, _ = _size([pb], [70000], tile_bytes=1 << 40)
    assert rc == 0
    assert N.load().fbsde_workspace_size(ctypes.byref(pb.c()), 70000, 0, ctypes.byref(ctypes.c_size_t())) == N.EINVAL
