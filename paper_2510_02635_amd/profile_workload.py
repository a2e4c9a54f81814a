"""Run one solve of a named workload (and optionally a plain device copy of known size), for profilers.

The copy gives the calibration factor of the HBM byte counters: its kernel moves exactly `--copy-mib`
MiB in and out, so counter / expected scales the counters of the solve's kernels.

  python -m paper_2510_02635_amd.profile_workload --workload allen_cahn_d1000_P1024_M4096_N20 --prec fp32c \
      --copy-mib 1024
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (problem kwargs, x0 kind, points)
    "allen_cahn_d1000_P1024_M4096_N20": (dict(d=1000, M=4096, N=20, T=0.3, f_kind=1, fp=(1.0, 1.0, 0, 0), g_kind=1,
                                              gp=(0.4, 0, 0, 0), eps_h=1.0, ridge_rel=1e-3, seed=0, instance=1),
                                         "normal:0.5", 1024),
    "shared_allen_cahn_d10000_P4096_M2048_N20": (dict(d=10000, M=2048, N=20, T=0.3, f_kind=1, fp=(1.0, 1.0, 0, 0),
                                                      g_kind=1, gp=(0.4, 0, 0, 0), shared_dw=1, seed=0, instance=4),
                                                 "normal_over_sqrt_d", 4096),
    # the paper's Burgers runtime setting (d = 10^4, M = 100, dt = 0.003, T = 0.3) under the paper-literal
    # per-anchor scheme, 64 replicas of the point x0 = 0
    "literal_burgers_d10000_M100_N100_P64": (dict(d=10000, M=100, N=100, T=0.3, f_kind=3,
                                                  fp=(2 ** 0.5 / 10000, 10000 / 2 + 0.5, 0, 0), g_kind=4,
                                                  gp=(0.3, 0, 0, 0), eps_h=1.0, ridge_rel=1e-3, instance=6),
                                             "zeros", 64),
    # the same scheme under the geometric coefficient family mu = 0.05 x, sigma = 0.2 diag(x), x0 = 1
    "literal_geometric_hjb_d1000_M100_N50_P64": (dict(d=1000, M=100, N=50, T=0.5, f_kind=2, fp=(1.0, 0, 0, 0),
                                                      g_kind=2, gp=(1.0, 0, 0, 0), eps_h=1.0, ridge_rel=1e-3,
                                                      instance=7), "ones", 64),
}
LITERAL = ("literal_burgers_d10000_M100_N100_P64", "literal_geometric_hjb_d1000_M100_N50_P64")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="allen_cahn_d1000_P1024_M4096_N20", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="fp32c", choices=["fp32c", "fp64"])
    ap.add_argument("--copy-mib", type=int, default=0, help="also run a device copy of this many MiB")
    ap.add_argument("--adjoint", action="store_true", help="solve with the tape, then the reverse mode of sum_p u_p")
    ap.add_argument("--coef", default="", help="mu0,sigma0,mu1,sigma1: the affine diagonal coefficient family "
                                                "(scheme R per point) instead of constant coefficients")
    ap.add_argument("--coef-x0", type=float, default=0.03, help="with --coef: every point at this constant")
    args = ap.parse_args()
    import torch

    import paper_2510_02635_amd as F
    from paper_2510_02635_amd import workloads

    kw, xkind, P = WORKLOADS[args.workload]
    if args.workload in LITERAL:
        if "geometric" in args.workload:
            pb = F.Problem(**kw)
            x0 = torch.ones((P, kw["d"]), dtype=torch.float64, device="cuda")
            for _ in range(2):
                u, st, _, _ = F.solve_literal_geometric(pb, x0, 0.05, 0.2)
        else:
            gvec = torch.full((kw["d"],), 1.0 / kw["d"], dtype=torch.float64, device="cuda")
            pb = F.Problem(gvec=gvec, **kw)
            x0 = torch.zeros((P, kw["d"]), dtype=torch.float64, device="cuda")
            ws = torch.empty(F.literal_workspace_size(pb, P, stored=True), dtype=torch.uint8, device="cuda")
            for _ in range(2):   # every level's particles kept, as in the bench
                u, st, _, _ = F.solve_literal(pb, x0, ws=ws)
        torch.cuda.synchronize()
        print(f"{args.workload} fp64 (literal, 2 solves): u[0]={u[0].item():.12g} "
              f"nonzero status={int((st != 0).sum())}", flush=True)
        return
    pb = F.Problem(prec=F.F32C if args.prec == "fp32c" else F.F64, **kw)
    x0 = torch.tensor(workloads.points(xkind, P, kw["d"], 1), dtype=torch.float64, device="cuda")
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.coef:
        cf = [float(v) for v in args.coef.split(",")]
        x0 = torch.full((P, kw["d"]), args.coef_x0, dtype=torch.float64, device="cuda")
        ws = torch.empty(F.coef_workspace_size(pb, P, *cf, tape=args.adjoint), dtype=torch.uint8, device="cuda")
        u, g, st = F.solve_coef(pb, x0, *cf, ws=ws, tape=args.adjoint)
        if args.adjoint:
            F.solve_coef_backward(pb, x0, torch.ones(P, dtype=torch.float64, device="cuda"), ws, *cf)
    elif args.adjoint:
        ws = F.workspace(pb, P, tape=True)
        u, g, st = F.solve(pb, x0, tape=True, ws=ws)
        F.solve_backward(pb, x0, torch.ones(P, dtype=torch.float64, device="cuda"), ws)
    else:
        ws = F.workspace(pb, P)
        u, g, st = F.solve(pb, x0, ws=ws)
    torch.cuda.synchronize()
    head = f"{args.workload} {args.prec}: u[0]={u[0].item():.12g} nonzero status={int((st != 0).sum())}"
    if kw.get("shared_dw"):
        # the shared form solves its regressions directly (Cholesky): no CG products to count
        print(head, flush=True)
    else:
        # the rows the CG products streamed (device count; x d x element bytes = their algorithmic read bytes)
        rows = F.workspace_cg_rows(ws)
        esz = 4 if args.prec == "fp32c" else 8
        print(f"{head} cg rows streamed={rows} algorithmic CG bytes={rows * kw['d'] * esz}", flush=True)


if __name__ == "__main__":
    main()
