"""Host-side checks of the C ABI: the library loads and exports every symbol that include/fbsde.h
declares; argument validation happens on the host (no GPU needed for an error return)."""
import ctypes
import os
import re

import pytest

import paper_2510_02635_amd as F
from paper_2510_02635_amd import _native as N


def _declared(repo_root):
    text = open(os.path.join(repo_root, "include", "fbsde.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|size_t|const char\*)\s+(fbsde_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol(repo_root):
    lib = N.load()
    names = _declared(repo_root)
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(N.EXPORTED)


def test_struct_layout_matches_header():
    # the ctypes mirror of fbsde_problem: 24 + 16 + 8 + 8 + 64 + 8 + 16 + 8 + 8 + 8 + 8 + 8 + 8 = 192 bytes
    assert ctypes.sizeof(N.CProblem) == 192
    assert N.CProblem.seed.offset == 168 and N.CProblem.prec.offset == 184
    # fbsde_coef: two int32 and four doubles
    assert ctypes.sizeof(N.CCoef) == 40
    assert N.CCoef.mu0.offset == 8 and N.CCoef.sigma1.offset == 32


@pytest.mark.parametrize("bad", [dict(d=0), dict(M=1), dict(N=0), dict(T=0.0), dict(s=-1.0), dict(f_kind=7),
                                 dict(g_kind=9), dict(ridge_rel=0.0, M=10, d=20), dict(newton_iters=0),
                                 dict(prec=5), dict(eps_h=-1.0)])
def test_invalid_descriptors_rejected_on_host(bad):
    kw = dict(d=8, M=64, N=3, T=0.3)
    kw.update(bad)
    pb = F.Problem(**kw)
    size = ctypes.c_size_t(0)
    rc = N.load().fbsde_workspace_size(ctypes.byref(pb.c()), 4, 0, ctypes.byref(size))
    assert rc == N.EINVAL
    assert N.load().fbsde_strerror(rc).decode().startswith("invalid")


def test_state_pitch_and_workspace_growth():
    lib = N.load()
    for d, prec, ld in [(100, N.F64, 112), (1000, N.F64, 1008), (1000, N.F32C, 1024), (10000, N.F64, 10000)]:
        pb = F.Problem(d=d, M=256, N=4, T=0.3, prec=prec)
        assert lib.fbsde_state_ld(ctypes.byref(pb.c())) == ld
    pb = F.Problem(d=100, M=512, N=5, T=0.3)
    a, b = F.workspace_size(pb, 1), F.workspace_size(pb, 1, tape=True)
    assert b > a > 512 * 112 * 8
    assert F.workspace_size(pb, 8) > a


def test_missing_gvec_and_tiny_workspace():
    pb = F.Problem(d=4, M=16, N=2, T=0.3, g_kind=N.G_AFFINE)
    size = ctypes.c_size_t(0)
    assert N.load().fbsde_workspace_size(ctypes.byref(pb.c()), 1, 0, ctypes.byref(size)) == N.EINVAL
    pb = F.Problem(d=4, M=16, N=2, T=0.3)
    # a workspace that is too small is refused before any device pointer is touched
    rc = N.load().fbsde_solve(ctypes.byref(pb.c()), 1, ctypes.c_void_p(16), ctypes.c_void_p(16), None,
                              ctypes.c_void_p(16), ctypes.c_void_p(16), 8, 0, None, None)
    assert rc == N.ENOSPC


def test_graph_capture_refuses_the_host_polled_loop(monkeypatch):
    # with the diagnostic host-polled CG loop selected, the per-point form polls the host between CG launches
    # unless cg_fixed_iters > 0: refused before any HIP call, so this runs without a GPU (the default
    # device-side loop captures any descriptor)
    monkeypatch.setenv("FBSDE_CG_HOST_LOOP", "1")
    pb = F.Problem(d=8, M=64, N=2, T=0.3)
    h = ctypes.c_void_p()
    rc = N.load().fbsde_graph_capture(ctypes.byref(pb.c()), 2, 1, 1, None, 1, 1, 1 << 30, 0, ctypes.byref(h), None)
    assert rc == N.EINVAL and not h.value
    assert N.load().fbsde_graph_launch(None, None) == N.EINVAL
    assert N.load().fbsde_graph_destroy(None) == 0


def test_autotune_validation_and_reset_on_host():
    shared = F.Problem(d=8, M=64, N=2, T=0.3, shared_dw=1)
    r = N.CTuneResult()
    assert N.load().fbsde_autotune(ctypes.byref(shared.c()), 2, 1, 1, 1 << 30, ctypes.byref(r), None) == N.EINVAL
    pb = F.Problem(d=8, M=64, N=2, T=0.3)
    assert N.load().fbsde_autotune(ctypes.byref(pb.c()), 0, 1, 1, 1 << 30, ctypes.byref(r), None) == N.EINVAL
    assert N.load().fbsde_autotune_reset() == 0


def test_size_limits_on_host():
    # the widest rows each precision supports and the most points one call takes are accepted; one more is not
    lib = N.load()
    size = ctypes.c_size_t(0)
    for prec, dmax in [(N.F64, 16384), (N.F32C, 32768)]:
        for d, ok in [(dmax, True), (dmax + 1, False)]:
            pb = F.Problem(d=d, M=64, N=2, T=0.3, prec=prec)
            rc = lib.fbsde_workspace_size(ctypes.byref(pb.c()), 2, 0, ctypes.byref(size))
            assert (rc == 0) == ok, (prec, d, rc)
    pb = F.Problem(d=4, M=16, N=2, T=0.3)
    assert lib.fbsde_workspace_size(ctypes.byref(pb.c()), 65535, 0, ctypes.byref(size)) == 0
    assert lib.fbsde_workspace_size(ctypes.byref(pb.c()), 65536, 0, ctypes.byref(size)) == N.EINVAL
    assert lib.fbsde_workspace_size(ctypes.byref(pb.c()), -1, 0, ctypes.byref(size)) == N.EINVAL
    # the batched call tiles an instance larger than one call
    cps = (N.CProblem * 1)(pb.c())
    Ps = (ctypes.c_int64 * 1)(70000)
    opts = N.CBatchOpts(N.BATCH_TILED, 2, 0, 512, 0)
    assert lib.fbsde_batched_workspace_size(cps, 1, ctypes.cast(Ps, ctypes.c_void_p), ctypes.byref(opts), 0,
                                            ctypes.byref(size)) == 0
    assert size.value > 0


def test_launch_timer_validation_on_host():
    lib = N.load()
    n = ctypes.c_int64(-1)
    assert lib.fbsde_launch_timer(2) == N.EINVAL
    assert lib.fbsde_launch_timer_read(None, None, -1, ctypes.byref(n)) == N.EINVAL
    assert lib.fbsde_launch_timer_read(None, None, 4, ctypes.byref(n)) == N.EINVAL
    # starting and stopping an empty record makes no HIP call
    assert lib.fbsde_launch_timer(1) == 0 and lib.fbsde_launch_timer(0) == 0
    assert lib.fbsde_launch_timer_read(None, None, 0, ctypes.byref(n)) == 0 and n.value == 0
    assert lib.fbsde_launch_timer_kinds(None, 0, ctypes.byref(n)) == 0 and n.value == 0
    assert lib.fbsde_launch_timer_kinds(None, 2, ctypes.byref(n)) == N.EINVAL
    assert lib.fbsde_launch_timer_kinds(None, 0, None) == N.EINVAL


def test_literal_scheme_validation_on_host():
    lib = N.load()
    size = ctypes.c_size_t(0)
    ok = F.Problem(d=100, M=200, N=4, T=0.3)
    assert lib.fbsde_literal_workspace_size(ctypes.byref(ok.c()), 3, ctypes.byref(size)) == N.OK
    # state W [P][M][ld], two Y buffers, the Gram matrices and row sums
    assert size.value >= 3 * 200 * (112 + 200 + 3) * 8
    for bad in (dict(M=257), dict(prec=N.F32C), dict(ridge_rel=0.0, M=300, d=8), dict(ridge_rel=0.0),
                dict(shared_dw=1)):
        kw = dict(d=100, M=200, N=4, T=0.3)
        kw.update(bad)
        pb = F.Problem(**kw)
        assert lib.fbsde_literal_workspace_size(ctypes.byref(pb.c()), 3, ctypes.byref(size)) == N.EINVAL, bad
    assert lib.fbsde_literal_workspace_size(ctypes.byref(ok.c()), 3, None) == N.EINVAL
    assert lib.fbsde_literal_workspace_size(ctypes.byref(ok.c()), 0, ctypes.byref(size)) == N.OK
    small, full = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.fbsde_literal_workspace_size(ctypes.byref(ok.c()), 3, ctypes.byref(small)) == N.OK
    assert lib.fbsde_literal_workspace_size_stored(ctypes.byref(ok.c()), 3, ctypes.byref(full)) == N.OK
    assert full.value >= small.value + 4 * 3 * 200 * 112 * 8   # N + 1 = 5 levels instead of one
    # P = 0: nothing to do, null pointers accepted; k_stop outside [0, N) and missing buffers rejected
    c = ctypes.byref(ok.c())
    assert lib.fbsde_solve_literal(c, 0, 0, None, None, None, None, None, None, 0, None) == N.OK
    for k_stop in (-1, 4):
        assert lib.fbsde_solve_literal(c, 1, k_stop, None, None, None, None, None, None, 0, None) == N.EINVAL
    assert lib.fbsde_solve_literal(c, 1, 0, None, None, None, None, None, None, 0, None) == N.EINVAL


def test_literal_coef_validation_on_host():
    lib = N.load()
    size = ctypes.c_size_t(0)
    pb = F.Problem(d=20, M=30, N=5, T=0.3)
    ok = N.CCoef(N.COEF_GEOMETRIC, 0, 0.1, 0.4)
    assert lib.fbsde_literal_coef_workspace_size(ctypes.byref(pb.c()), ctypes.byref(ok), 2, ctypes.byref(size)) == N.OK
    # every level's displacements are kept: (N + 1) P M ld doubles at least
    assert size.value >= 6 * 2 * 30 * 32 * 8
    for bad in (N.CCoef(0, 0, 0.1, 0.4), N.CCoef(N.COEF_GEOMETRIC, 1, 0.1, 0.4), N.CCoef(N.COEF_GEOMETRIC, 0, 0.1, 0.0),
                N.CCoef(N.COEF_GEOMETRIC, 0, float("nan"), 0.4)):
        assert lib.fbsde_literal_coef_workspace_size(ctypes.byref(pb.c()), ctypes.byref(bad), 2,
                                                     ctypes.byref(size)) == N.EINVAL
    assert lib.fbsde_literal_coef_workspace_size(ctypes.byref(pb.c()), None, 2, ctypes.byref(size)) == N.EINVAL
    # the geometric kind takes no affine parts; the affine diagonal kind takes additive noise alone
    geo_aff = N.CCoef(N.COEF_GEOMETRIC, 0, 0.1, 0.4, 0.2, 0.0)
    assert lib.fbsde_literal_coef_workspace_size(ctypes.byref(pb.c()), ctypes.byref(geo_aff), 2,
                                                 ctypes.byref(size)) == N.EINVAL
    ou = N.CCoef(N.COEF_AFFINE_DIAG, 0, -0.8, 0.0, 0.2, 0.5)
    assert lib.fbsde_literal_coef_workspace_size(ctypes.byref(pb.c()), ctypes.byref(ou), 2, ctypes.byref(size)) == N.OK
    flat = N.CCoef(N.COEF_AFFINE_DIAG, 0, -0.8, 0.0, 0.2, 0.0)
    assert lib.fbsde_literal_coef_workspace_size(ctypes.byref(pb.c()), ctypes.byref(flat), 2,
                                                 ctypes.byref(size)) == N.EINVAL
    c = ctypes.byref(pb.c())
    assert lib.fbsde_solve_literal_coef(c, ctypes.byref(ok), 0, 0, None, None, None, None, None, None, 0, None) == N.OK
    assert lib.fbsde_solve_literal_coef(c, ctypes.byref(ok), 1, 5, None, None, None, None, None, None, 0, None) == N.EINVAL
