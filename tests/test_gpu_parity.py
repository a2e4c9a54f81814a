"""GPU parity of the HIP path against the FP64 oracle on identical seeded inputs.

Bar (tolerances of the scheme's precision modes): FP64 relative error <= 1e-10 on u and on
grad u (norm-wise over a point's d coordinates); FP32C <= 1e-5 against the FP64 oracle; Philox
words bit-exact; normals within a few ulp (the two sides use different libm log / sincos).
Sizes span several blocks per point, ragged row chunks (M not a multiple of the block's rows),
d not a multiple of the 4-coordinate groups, and every team width (1 .. 16 waves per row).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2510_02635_amd as F  # noqa: E402
from oracle import philox as OP  # noqa: E402
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


def _x0(kind, P, d, seed):
    return workloads.points(kind, P, d, seed)


def _run_solve(hp, op, x0, tol_u, tol_g, points=None):
    _say(f"[solve] d={hp.d} M={hp.M} N={hp.N} P={x0.shape[0]} prec={hp.prec} f={hp.f_kind} g={hp.g_kind}")
    xt = torch.tensor(x0, dtype=torch.float64, device=DEV)
    u, g, st, iters = F.solve(hp, xt, return_iters=True)
    torch.cuda.synchronize()
    u, g, st = u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    idx = range(x0.shape[0]) if points is None else points
    for p in idx:
        ref = OS.solve_point(op, x0[p], p)
        eu = abs(u[p] - ref["u"]) / max(abs(ref["u"]), 1e-300)
        eg = rel_err(g[p], ref["grad"])
        _say(f"  p={p} u={u[p]:.12g} ref={ref['u']:.12g} rel_u={eu:.2e} rel_grad={eg:.2e} cg={iters}")
        assert st[p] == ref["status"] == 0
        assert eu <= tol_u, (p, eu)
        assert eg <= tol_g, (p, eg)
    return iters


def test_philox_words_and_normals_match_oracle():
    hp, op = problems(d=37, M=16, N=3, T=0.3, seed=0xDEADBEEF12345, instance=9, point_base=5)
    out, words = F.normals(hp, 2, 1, 3, 10)
    torch.cuda.synchronize()
    ref_w = OP.raw_words(op.seed, op.instance, 7, 1, np.arange(3, 13), (37 + 3) // 4)
    assert np.array_equal(words.cpu().numpy().view(np.uint32), ref_w)
    ref = OP.normals(op.seed, op.instance, 7, 1, 13, 37)[3:13]
    got = out.cpu().numpy()
    # the kernels reduce the angle 2 pi u exactly in integers; the oracle rounds 2 pi u first, which
    # moves its sin / cos by up to ~1e-15 absolute near the zero crossings
    ulp = np.abs(got - ref) / np.spacing(np.maximum(np.abs(ref), 1e-300))
    assert np.max(np.abs(got - ref)) < 4e-15
    assert np.median(ulp) <= 2.0


def test_fp32c_normals_match_oracle_to_fp32_rounding():
    """FP32C draws its normals in FP32 (integer-reduced logarithm for the radius, Taylor sin/cos on the
    exactly reduced angle): 2^17 normals within 8 FP32 ulps of the FP64 oracle, with nothing lost as
    u -> 1 (small radii) or u -> 0 (the tail)."""
    hp, op = problems(d=1024, M=16, N=3, T=0.3, seed=0x5EED, instance=3, prec=F.F32C)
    out, words = F.normals(hp, 0, 2, 0, 128)
    torch.cuda.synchronize()
    ref = OP.normals(op.seed, op.instance, op.point_base, 2, 128, 1024)
    got = out.cpu().numpy()
    ulp32 = np.spacing(np.maximum(np.abs(ref), 1e-30).astype(np.float32)).astype(np.float64)
    err = np.abs(got - ref)
    _say(f"[normals fp32c] max abs {err.max():.2e}, max ulps {np.max(err / ulp32):.2f}, median ulps "
         f"{np.median(err / ulp32):.2f}")
    assert np.max(err) < 4e-6
    assert np.max(err / np.maximum(ulp32, 1e-7)) <= 8.0


@pytest.mark.parametrize("d,M,prec", [(37, 100, F.F64), (1000, 96, F.F64), (3000, 20, F.F32C), (10000, 8, F.F64)])
def test_terminal_matches_oracle(d, M, prec):
    hp, op = problems(d=d, M=M, N=3, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                      gp=(0.4, 0, 0, 0), prec=prec, seed=3)
    x0 = _x0("normal:0.5", 2, d, 1)
    _say(f"[terminal] d={d} M={M} prec={prec}")
    W, Y, st = F.terminal(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    tol = 1e-13 if prec == F.F64 else 1e-6
    for p in range(2):
        Wr = OS.brownian_path(op, p)[op.N]
        assert rel_err(W[p, :, :d].double().cpu().numpy(), Wr) < tol
        assert np.all(W[p, :, d:].cpu().numpy() == 0.0)
        Yr, _, _ = OS.g_eval(op, OS.positions(op, x0[p], Wr, op.N))
        assert rel_err(Y[p].cpu().numpy(), Yr) < tol
    assert np.all(st.cpu().numpy() == 0)


@pytest.mark.parametrize("d,M,k,f_kind,g_kind", [(37, 100, 1, F.F_ALLEN_CAHN, F.G_AC), (600, 257, 0, F.F_HJB,
                                                                                       F.G_HJB_LOG),
                                                 (1500, 50, 2, F.F_ZERO, F.G_QUAD)])
def test_solve_step_matches_oracle_level(d, M, k, f_kind, g_kind):
    N = 3
    hp, op = problems(d=d, M=M, N=N, T=0.3, f_kind=f_kind, fp=(1.0, 1.0, 0, 0), g_kind=g_kind, gp=(0.4, 0, 0, 0),
                      seed=11, eps_h=1.0, ridge_rel=1e-3)
    x0 = _x0("normal:0.3", 2, d, 2)
    _say(f"[step] d={d} M={M} k={k}")
    ld = F.state_ld(hp)
    W = torch.zeros((2, M, ld), dtype=torch.float64, device=DEV)
    Ynext = torch.zeros((2, M), dtype=torch.float64, device=DEV)
    paths, refs = [], []
    rng = np.random.default_rng(4)
    for p in range(2):
        path = OS.brownian_path(op, p)
        Yn = np.sin(path[k + 1].sum(1)) + 0.1 * rng.standard_normal(M)   # any response works for one level
        W[p, :, :d] = torch.tensor(path[k + 1], device=DEV)
        Ynext[p] = torch.tensor(Yn, device=DEV)
        paths.append(path)
        refs.append(OS.level_step(op, k, path[k + 1], path[k], Yn))
    Y, a, ax, st = F.solve_step(hp, k, W, Ynext)
    torch.cuda.synchronize()
    for p in range(2):
        r = refs[p]
        assert abs(a[p].item() - r["alpha"]) <= 1e-10 * max(1.0, abs(r["alpha"]))
        assert rel_err(ax[p].cpu().numpy(), r["alpha_x"]) <= 1e-10
        assert rel_err(Y[p].cpu().numpy(), r["Y"]) <= 1e-10
        assert rel_err(W[p, :, :d].cpu().numpy(), paths[p][k]) <= 1e-13 or k == 0
        if k == 0:
            assert torch.all(W[p] == 0)
    assert np.all(st.cpu().numpy() == 0)


CASES = [
    # (name, problem kwargs, x0 kind, P)
    ("allen_cahn_d100", dict(d=100, M=512, N=5, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                             gp=(0.4, 0, 0, 0)), "zero", 1),
    ("hjb_ragged_d37_mu", dict(d=37, M=100, N=3, T=0.5, f_kind=F.F_HJB, fp=(0.8, 0, 0, 0), g_kind=F.G_HJB_LOG,
                               gp=(1.0, 0, 0, 0), seed=7), "uniform", 3),
    ("heat_d1000", dict(d=1000, M=300, N=2, T=0.3, f_kind=F.F_ZERO, g_kind=F.G_QUAD), "normal:0.5", 2),
    ("ac_d600_team1_q4", dict(d=600, M=130, N=2, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                              gp=(0.4, 0, 0, 0)), "normal:0.2", 2),
    ("ac_d1500_team2", dict(d=1500, M=70, N=2, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                            gp=(0.4, 0, 0, 0)), "normal:0.2", 2),
    ("hjb_d3000_team4", dict(d=3000, M=64, N=2, T=1.0, f_kind=F.F_HJB, fp=(1.3, 0, 0, 0), g_kind=F.G_HJB_LOG,
                             gp=(1.0, 0, 0, 0)), "uniform", 2),
    ("ac_d5000_team8", dict(d=5000, M=50, N=2, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                            gp=(0.4, 0, 0, 0)), "normal_over_sqrt_d", 1),
    ("ac_d10000_team16", dict(d=10000, M=40, N=2, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                              gp=(0.4, 0, 0, 0)), "normal_over_sqrt_d", 1),
    ("uniform_weights_d64", dict(d=64, M=200, N=4, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(0.5, 2.0, 0, 0),
                                 g_kind=F.G_HJB_LOG, gp=(0.6, 0, 0, 0), eps_h=0.0, ridge_rel=0.0), "normal:0.3", 2),
    # Burgers-type family with the logistic terminal (fp0 = s/d, fp1 = d/s^2 + 1/2, gvec = 1/d)
    ("burgers_logistic_d50", dict(d=50, M=300, N=3, T=0.5, f_kind=F.F_BURGERS, fp=(2 ** 0.5 / 50, 25.5, 0, 0),
                                  g_kind=F.G_LOGISTIC, gp=(0.5, 0, 0, 0), gvec=np.ones(50) / 50), "normal:0.5", 3),
    ("burgers_logistic_d400_M120", dict(d=400, M=120, N=2, T=0.5, f_kind=F.F_BURGERS,
                                        fp=(2 ** 0.5 / 400, 200.5, 0, 0), g_kind=F.G_LOGISTIC, gp=(0.5, 0, 0, 0),
                                        gvec=np.linspace(-1.0, 2.0, 400) / 400), "normal:0.5", 2),
]


@pytest.mark.parametrize("name,kw,xkind,P", CASES, ids=[c[0] for c in CASES])
def test_solve_fp64_matches_oracle(name, kw, xkind, P):
    mu = None
    if "mu" in name:
        mu = 0.3 * np.cos(np.arange(kw["d"]))
    hp, op = problems(mu=mu, **kw)
    _run_solve(hp, op, _x0(xkind, P, kw["d"], 5), 1e-10, 1e-10)


FP32C_CASES = CASES[:3] + CASES[5:6] + CASES[9:11]


@pytest.mark.parametrize("name,kw,xkind,P", FP32C_CASES, ids=[c[0] for c in FP32C_CASES])
def test_solve_fp32c_matches_fp64_oracle(name, kw, xkind, P):
    mu = None
    if "mu" in name:
        mu = 0.3 * np.cos(np.arange(kw["d"]))
    hp, op = problems(mu=mu, prec=F.F32C, **kw)
    _run_solve(hp, op, _x0(xkind, P, kw["d"], 5), 1e-5, 1e-5)


def test_affine_closed_form_on_gpu():
    d, M, N, T, c1, b = 24, 96, 5, 0.5, 0.7, 0.4
    rng = np.random.default_rng(3)
    a = rng.standard_normal(d)
    mu = 0.2 * rng.standard_normal(d)
    hp, op = problems(mu=mu, gvec=a, d=d, M=M, N=N, T=T, s=1.3, f_kind=F.F_ALLEN_CAHN, fp=(c1, 0, 0, 0),
                      g_kind=F.G_AFFINE, gp=(b, 0, 0, 0), ridge_rel=0.0, seed=2)
    x0 = rng.standard_normal((3, d))
    _say("[affine closed form]")
    u, g, st = F.solve(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    fac = (1 - c1 * T / N) ** N
    for p in range(3):
        ue = (a @ (x0[p] + mu * T) + b) / fac
        assert abs(u[p].item() - ue) <= 1e-11 * max(1, abs(ue))
        assert rel_err(g[p].cpu().numpy(), a / fac) <= 1e-11


def _extreme_words():
    """Philox words that counters rarely produce, in quadruples (radius word, angle word, radius, angle)."""
    rad = {0, 1, 2, 3, 4, 5, 0xFFFFFFFF, 0xFFFFFFFE, 0xFFFFFFFD, 0x7FFFFFFF, 0x80000000, 0x80000001, 0x55555555}
    for e in range(32):
        rad.update({(1 << e) - 1, 1 << e, (1 << e) + 1})
        s = int(math.floor(math.sqrt(2.0) * (1 << e)))          # the mantissa switch at sqrt(2)
        rad.update(range(max(s - 2, 0), s + 3))
    rad = sorted(v for v in rad if 0 <= v <= 0xFFFFFFFF)
    ang = {0, 1, 2, 0xFFFFFFFF, 0xFFFFFFFE}
    for k in range(8):                                         # octant boundaries
        ang.update(((k << 29) + dv) % (1 << 32) for dv in (-2, -1, 0, 1, 2))
    ang = sorted(ang)
    rng = np.random.default_rng(17)
    rad += [int(v) for v in rng.integers(0, 1 << 32, 64, dtype=np.uint64)]
    ang += [int(v) for v in rng.integers(0, 1 << 32, 32, dtype=np.uint64)]
    quads = [(r, ang[i % len(ang)], rad[(i + 1) % len(rad)], ang[(7 * i + 3) % len(ang)]) for i, r in enumerate(rad)]
    quads += [(0x55555555, a, 0xFFFFFFFF, a) for a in ang]
    return np.array(quads, dtype=np.uint64)


def _box_muller_mp(quads):
    """Reference normals at 40 significant digits (independent of both the oracle's FP64 and the kernels)."""
    import mpmath
    mpmath.mp.dps = 40
    out = np.zeros(quads.shape, dtype=np.float64)
    two32 = mpmath.mpf(2) ** 32
    for n, (a, b, c, d) in enumerate(quads.tolist()):
        for slot, (wr, wa) in enumerate(((a, b), (c, d))):
            r = mpmath.sqrt(-2 * mpmath.log((wr + mpmath.mpf("0.5")) / two32))
            t = 2 * mpmath.pi * (wa + mpmath.mpf("0.5")) / two32
            out[n, 2 * slot] = float(r * mpmath.cos(t))
            out[n, 2 * slot + 1] = float(r * mpmath.sin(t))
    return out


@pytest.mark.parametrize("prec,bits,max_ulps", [(F.F64, 52, 16.0), (F.F32C, 23, 8.0)], ids=["fp64", "fp32c"])
def test_box_muller_at_extreme_words(prec, bits, max_ulps):
    """The transform at u -> 0 (w = 0: the largest radius), u -> 1 (w = 2^32 - 1: radius ~1.5e-5), every power of
    two and the sqrt(2) switch of the logarithm's reduction, and angles at the eight octant boundaries, against a
    40-digit reference: every component within `max_ulps` units in the last place of its own magnitude."""
    quads = _extreme_words()
    ref = _box_muller_mp(quads)
    words = torch.tensor(quads.astype(np.uint32).view(np.int32), device=DEV)
    got = F.box_muller(words, prec).cpu().numpy()
    ulp = np.exp2(np.floor(np.log2(np.abs(ref))) - bits)
    err = np.abs(got - ref) / ulp
    i = np.unravel_index(np.argmax(err), err.shape)
    _say(f"[box-muller extremes] prec={prec} {quads.shape[0]} quadruples, max {err.max():.2f} ulps at words "
         f"{quads[i[0]].tolist()} slot {i[1]}, median {np.median(err):.2f}")
    assert np.all(np.isfinite(got))
    assert err.max() <= max_ulps
