#!/usr/bin/env python3
"""Benchmark of the localized FBSDE-LLR hot path on one MI355X.

Workload (one "step" = one full solve, Algorithm 1, of a batch of evaluation points):
  d = 1000, P = 1024 points x0 ~ N(0, 0.25 I_d), T = 0.3, N = 20 time steps, M = 4096 particles per point,
  Allen-Cahn f(u) = u - u^3 with g(x) = 1 / (2 + 0.4 |x|^2), sigma = sqrt(2) I, Gaussian kernel h = 1,
  ridge 1e-3, Newton 8 iterations, Philox seed 0 / instance 1.
Headline value: solved points per second (u and grad u) in the FP32-compensated mode; the FP64 mode is
timed beside it, and both are compared with the FP64 oracle on sample points.

Extra objects on the JSON line:
  roofline      -- the device-side CG loop (the dominant kernel: one launch solves a level's CG for every
                   point, each iteration one fused read of the point's state), HBM-bound: algorithmic
                   bytes per launch (the rows its products streamed, counted on the device, x d x 4 B) /
                   its average launch time measured here with HIP events on the library's stream.
  cpu_baseline  -- the FP64 oracle timed on this host's cores on a bounded sample of points.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline] [--skip-fp64]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
METRIC = "solved points/sec (u,∇u) + fwd+adjoint points/sec at d=1000, rel err vs FP64"
KERNEL_SRCS = [os.path.join(ROOT, "paper_2510_02635_amd", "csrc", f)
               for f in ("fbsde_cgloop.hpp", "fbsde_rowteam.hpp", "fbsde_device.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cg_loop_d1000_P1024_M4096_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(F, prec):
    return F.Problem(d=1000, M=4096, N=20, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0.0, 0.0), g_kind=F.G_AC,
                     gp=(0.4, 0.0, 0.0, 0.0), eps_h=1.0, ridge_rel=1e-3, newton_iters=8, seed=0, instance=1,
                     prec=prec)


def kernel_source_hash():
    """Hash of the sources of the CG loop kernel; the stored counter traffic is used only if it matches."""
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def timed_solves(F, torch, pb, x0, ws, warmup, steps, loop=None):
    """Seconds per solve over `steps` timed solves after `warmup` untimed ones (no host wait inside the
    timed region).  With a dict in `loop`, the library's launch timer records the CG loop launches of the
    timed solves (HIP events on the launching stream): loop["ms"] gets their durations and loop["rows"]
    the particle rows their products streamed in one solve (every timed solve is the same solve).  The
    per-level iteration counts come from one more solve after the timed region."""
    for _ in range(warmup):
        F.solve(pb, x0, ws=ws)
    torch.cuda.synchronize()
    if loop is not None:
        F.launch_timer(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        u, g, st = F.solve(pb, x0, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if loop is not None:
        F.launch_timer(False)
        ms = F.launch_timer_read()
        kinds = F.launch_timer_kinds()
        loop["ms"] = ms[kinds == F.TIMED_CG_LOOP].tolist()
        loop["rows"] = F.workspace_cg_rows(ws)
    iters = F.solve(pb, x0, ws=ws, return_iters=True)[3]
    return dt / steps, u, g, st, iters


def loop_roofline(loop, steps, d, esz):
    """The CG loop launches of the timed solves: algorithmic bytes (rows streamed x d x element bytes) per
    launch over the average launch duration."""
    import numpy as np
    ms = np.asarray(loop["ms"], dtype=np.float64)
    per_solve = ms.size // max(steps, 1)
    alg = loop["rows"] * d * esz / max(per_solve, 1)
    return {"avg_launch_ms": float(ms.mean()), "launches": int(ms.size), "algorithmic_bytes_per_launch": float(alg),
            "achieved": alg / (ms.mean() * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=3, help="oracle points timed for the CPU baseline")
    ap.add_argument("--no-shared", action="store_true", help="skip the shared-increment (MFMA) leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-instance leg")
    ap.add_argument("--batched-points", type=int, default=8, help="points per instance in the batched leg")
    ap.add_argument("--no-small", action="store_true", help="skip the one-point and d = 10^4 adjoint legs")
    ap.add_argument("--no-literal", action="store_true", help="skip the paper-literal per-anchor leg")
    ap.add_argument("--batched-full-forward", action="store_true",
                    help="also run the batched workload at its configured 256 points per instance, forward, in "
                         "slices of 8 instances (several minutes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the points of this workload are independent, so a multi-GPU run "
              f"would shard them with no exchange; --gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_02635_amd as F
    from paper_2510_02635_amd import workloads

    F._native.load()
    dev = "cuda"
    P = args.points
    x0_np = workloads.points("normal:0.5", P, 1000, seed=1)
    x0 = torch.tensor(x0_np, dtype=torch.float64, device=dev)
    out = {}

    # ---------------- FP32C (headline)
    pb32 = workload(F, F.F32C)
    ws32 = F.workspace(pb32, P, device=dev)
    log(f"[bench] fp32c: workspace {ws32.numel() / 2**30:.1f} GiB")
    loop32 = {}
    sec32, u32, g32, st32, it32 = timed_solves(F, torch, pb32, x0, ws32, args.warmup, args.steps, loop32)
    log(f"[bench] fp32c: {sec32 * 1e3:.1f} ms/solve, cg iterations per level {it32}")
    # the read ceiling on the same buffer: a plain stream over the whole [P][M][ld] state
    rd32_ms = F.time_kernel(pb32, P, "stream_read", ws32, reps=6)
    ld32 = F.state_ld(pb32)
    rev32_ms = F.time_kernel(pb32, P, "reverse_newton", ws32, reps=3)
    u32, g32, st32 = u32.cpu().numpy(), g32.cpu().numpy(), st32.cpu().numpy()
    del ws32
    torch.cuda.empty_cache()

    # ---------------- FP32C forward (with tape) + adjoint of L = sum_p u_p
    wsa = F.workspace(pb32, P, tape=True, device=dev)
    ubar = torch.ones(P, dtype=torch.float64, device=dev)

    def fwd_adj():
        F.solve(pb32, x0, tape=True, ws=wsa)
        return F.solve_backward(pb32, x0, ubar, wsa)

    for _ in range(args.warmup):
        fwd_adj()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x0bar, gpbar, fpbar, sta = fwd_adj()
    torch.cuda.synchronize()
    sec_fa = (time.perf_counter() - t0) / args.steps
    # the iteration counts of both passes, from one more forward + backward after the timed region
    it_fwd_tape = F.solve(pb32, x0, tape=True, ws=wsa, return_iters=True)[3]
    it_adj = F.solve_backward(pb32, x0, ubar, wsa, return_iters=True)[4]
    log(f"[bench] fp32c fwd+adj: {sec_fa * 1e3:.1f} ms per solve + backward")
    x0bar = x0bar.cpu().numpy()
    del wsa
    torch.cuda.empty_cache()

    # ---------------- FP64: at the oracle-parity tolerance (1e-13), and at FP32C's tolerance (1e-7) for the
    # speedup at equal accuracy
    sec64 = sec64e = None
    u64 = g64 = u64e = g64e = None
    loop64 = None
    it64 = it64e = None
    if not args.skip_fp64:
        pb64 = workload(F, F.F64)
        ws64 = F.workspace(pb64, P, device=dev)
        log(f"[bench] fp64: workspace {ws64.numel() / 2**30:.1f} GiB")
        loop64 = {}
        sec64, u64, g64, st64, it64 = timed_solves(F, torch, pb64, x0, ws64, min(args.warmup, 1), args.steps, loop64)
        log(f"[bench] fp64: {sec64 * 1e3:.1f} ms/solve, cg iterations per level {it64}")
        u64, g64 = u64.cpu().numpy(), g64.cpu().numpy()
        pb64e = workload(F, F.F64)
        pb64e.cg_rtol = 1e-7
        sec64e, u64e, g64e, _, it64e = timed_solves(F, torch, pb64e, x0, ws64, min(args.warmup, 1), args.steps)
        log(f"[bench] fp64 at cg_rtol 1e-7: {sec64e * 1e3:.1f} ms/solve, cg iterations per level {it64e}")
        u64e, g64e = u64e.cpu().numpy(), g64e.cpu().numpy()
        del ws64
        torch.cuda.empty_cache()

    # ---------------- roofline of the dominant kernel: the device-side CG loop (every CG iteration of every
    # point of a level in one launch; each iteration one fused read of the point's state)
    d, M = 1000, 4096
    lr32 = loop_roofline(loop32, args.steps, d, 4)
    achieved32 = lr32["achieved"]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_source_sha256_16") == kernel_source_hash():
            traffic = tr.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved32, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved32 / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_cg_loop<float, float, 4, 1> (a level's whole CG solve; one fused state read per iteration)",
                "algorithmic_bytes_per_launch": round(lr32["algorithmic_bytes_per_launch"]),
                "avg_launch_ms": round(lr32["avg_launch_ms"], 4),
                "launches": {"timed_region": "the CG loop launches of the timed solves, HIP events on their stream",
                             "recorded": lr32["launches"],
                             "bytes": "rows streamed by the products of one solve (device count) x d x 4 B, over "
                                      "its 20 launches"}}
    ceiling = P * M * ld32 * 4 / (rd32_ms * 1e-3) / 1e9
    roofline["read_ceiling"] = {"kernel": "k_stream_read (16-byte non-temporal loads over the same state, nothing else)",
                                "bytes_per_launch": P * M * ld32 * 4, "avg_launch_ms": round(rd32_ms, 4),
                                "achieved": round(ceiling, 1), "frac_of_peak": round(ceiling / HBM_PEAK_GBS, 4),
                                "cg_loop_frac_of_ceiling": round(achieved32 / ceiling, 4)}
    if loop64:
        lr64 = loop_roofline(loop64, args.steps, d, 8)
        roofline["fp64_kernel"] = {"achieved": round(lr64["achieved"], 1), "avg_launch_ms": round(lr64["avg_launch_ms"], 4),
                                   "algorithmic_bytes_per_launch": round(lr64["algorithmic_bytes_per_launch"]),
                                   "frac": round(lr64["achieved"] / HBM_PEAK_GBS, 4)}

    # ---------------- whole-job state traffic: passes over the [P][M][d] state per solve
    # forward: 1 write (terminal sweep), per level 1 moments read + K_k CG reads + reversal read and
    # write (read only at k = 0); adjoint: per level advance read and write + K'_k CG reads + 1 row-dot
    # read (+ 1 warm-start product from the second level on), then 1 terminal read.  [P][M] FP64 side
    # arrays (weights, Y) are below 0.3 % and not counted; the row pitch beyond d is not counted either.
    def fwd_passes(iters):
        return 1 + sum(1 + k + 2 for k in iters) - 1

    def adj_passes(iters):
        # + one CG product per warm-started level (k > 0; the design has full rank here, M > d + 1)
        return sum(3 + k for k in iters) + 1 + (len(iters) - 1)

    state32 = P * M * d * 4
    state64 = P * M * d * 8

    def whole(passes, state, sec):
        gbs = passes * state / sec / 1e9
        return {"state_passes": passes, "bytes": passes * state, "achieved_GBs": round(gbs, 1),
                "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}

    whole_job = {"fp32c_forward": whole(fwd_passes(it32), state32, sec32),
                 "fp32c_fwd_adj": whole(fwd_passes(it_fwd_tape) + adj_passes(it_adj), state32, sec_fa)}
    if sec64:
        whole_job["fp64_forward"] = whole(fwd_passes(it64), state64, sec64)
        whole_job["fp64_forward_rtol1e-7"] = whole(fwd_passes(it64e), state64, sec64e)

    # ---------------- oracle: CPU baseline and errors on sample points
    cpu = None
    errs = {}
    if not args.no_cpu_baseline:
        from oracle import scheme as OS
        try:
            from threadpoolctl import threadpool_info
            threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
        except Exception:   # threadpoolctl missing: the BLAS default is every core
            threads = os.cpu_count()
        op = OS.Problem(d=1000, M=4096, N=20, T=0.3, f_kind=OS.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=OS.G_AC,
                        gp=(0.4, 0, 0, 0), eps_h=1.0, ridge_rel=1e-3, newton_iters=8, seed=0, instance=1)
        n = max(1, args.cpu_sample)
        t0 = time.perf_counter()
        refs = [OS.solve_point(op, x0_np[p], p) for p in range(n)]
        tcpu = time.perf_counter() - t0
        model = None
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
        except OSError:
            pass
        cpu = {"value": round(n / tcpu, 5), "unit": "points/s", "cores": int(threads), "kind": "oracle",
               "sample": f"points 0..{n - 1} of the {P}-point workload, full solve each ({tcpu:.1f} s)",
               "host": {"cpu_model": model, "logical_cpus": os.cpu_count()}}
        adj_ref = OS.adjoint_point(op, x0_np[0], 0, ubar=1.0)
        errs["fp32c_x0bar_point0"] = float(f"{np.linalg.norm(x0bar[0] - adj_ref['x0bar']) / np.linalg.norm(adj_ref['x0bar']):.3e}")
        for name, uu, gg in (("fp32c", u32, g32), ("fp64", u64, g64), ("fp64_rtol1e-7", u64e, g64e)):
            if uu is None:
                continue
            eu = max(abs(uu[p] - refs[p]["u"]) / abs(refs[p]["u"]) for p in range(n))
            eg = max(float(np.linalg.norm(gg[p] - refs[p]["grad"]) / np.linalg.norm(refs[p]["grad"]))
                     for p in range(n))
            errs[name] = {"u": float(f"{eu:.3e}"), "grad": float(f"{eg:.3e}")}

    # ---------------- the other single-GPU configurations: one point at d = 100 (latency-bound, no roofline
    # claim) and 128 points at d = 10^4 with M = 1024, forward + adjoint
    small = None
    if not args.no_small:
        small = {}
        pb0 = F.Problem(d=100, M=512, N=5, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC,
                        gp=(0.4, 0, 0, 0))
        x00 = torch.zeros((1, 100), dtype=torch.float64, device=dev)
        ws0 = F.workspace(pb0, 1, device=dev)
        for _ in range(3):
            F.solve(pb0, x00, ws=ws0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            F.solve(pb0, x00, ws=ws0)
        torch.cuda.synchronize()
        sec0 = (time.perf_counter() - t0) / 20
        # the same solve captured once into a HIP graph and replayed with one launch; the graph needs a fixed
        # number of CG launches per level (a converged point's launches exit at once)
        # the same solve captured once into a HIP graph (default CG settings: each level's CG is one loop
        # launch) and replayed with one launch
        cs0 = F.CapturedSolve(pb0, x00, want_grad=True)
        for _ in range(3):
            cs0.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            ug0, _, _ = cs0.launch()
        torch.cuda.synchronize()
        secg0 = (time.perf_counter() - t0) / 20
        ue0 = F.solve(pb0, x00, ws=ws0)[0]
        small["allen_cahn_d100_P1_M512_N5_fp64"] = {"ms_per_solve": round(sec0 * 1e3, 3),
                                                    "points_per_s": round(1.0 / sec0, 1),
                                                    "graph_replay_ms_per_solve": round(secg0 * 1e3, 3),
                                                    "graph_u_equals_eager": bool((ug0 == ue0).all().item()),
                                                    "bound": "launch latency (a 0.4 MB state)"}
        cs0.close()
        log(f"[bench] one point, d = 100: {sec0 * 1e3:.2f} ms per solve, {secg0 * 1e3:.2f} ms as a HIP graph replay")
        del ws0
        P3, d3, M3 = 128, 10000, 1024
        pb3 = F.Problem(d=d3, M=M3, N=20, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC,
                        gp=(0.4, 0, 0, 0), prec=F.F32C, instance=3)
        x3 = torch.tensor(workloads.points("normal_over_sqrt_d", P3, d3, seed=3), dtype=torch.float64, device=dev)
        ws3 = F.workspace(pb3, P3, tape=True, device=dev)
        ub3 = torch.ones(P3, dtype=torch.float64, device=dev)

        def fwd_adj3():
            F.solve(pb3, x3, tape=True, ws=ws3)
            F.solve_backward(pb3, x3, ub3, ws3)

        fwd_adj3()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fwd_adj3()
        torch.cuda.synchronize()
        sec3 = (time.perf_counter() - t0) / args.steps
        it3f = F.solve(pb3, x3, tape=True, ws=ws3, return_iters=True)[3]
        it3a = F.solve_backward(pb3, x3, ub3, ws3, return_iters=True)[4]
        state3 = P3 * M3 * d3 * 4
        # M <= d + 1: neither CG is warm-started, so the adjoint has no extra product per level
        passes3 = fwd_passes(it3f) + sum(3 + k for k in it3a) + 1
        small["allen_cahn_d10000_P128_M1024_N20_fp32c_fwd_adj"] = {
            "value": round(P3 / sec3, 2), "unit": "points/s", "ms_per_step": round(sec3 * 1e3, 3),
            "state_passes": passes3, "achieved_GBs": round(passes3 * state3 / sec3 / 1e9, 1),
            "frac_of_hbm_peak": round(passes3 * state3 / sec3 / 1e9 / HBM_PEAK_GBS, 4),
            "cg_iters_per_level": it3f, "adjoint_cg_iters_per_level": it3a}
        log(f"[bench] d = 10^4, 128 points fwd+adj: {sec3 * 1e3:.1f} ms")
        del ws3, x3
        # the Hamilton-Jacobi-type equation at the shape of the paper's runtime table (d = 500, T = 0.5,
        # M = 100, x = 0, dt = 0.0005 and dt / 2^4), 64 independent replicas of the point, FP64; its exact
        # solution at (0, 0) is 1
        hj = {}
        for Nh in (1000, 16000):
            pbh = F.Problem(d=500, M=100, N=Nh, T=0.5, f_kind=F.F_HJ_SINK, fp=(0.1, 0, 0, 0), g_kind=F.G_HJ_GAUSS,
                            gp=(0.5, 0, 0, 0), seed=0, instance=9)
            xh = torch.zeros((64, 500), dtype=torch.float64, device=dev)
            wsh = F.workspace(pbh, 64, device=dev)
            F.solve(pbh, xh, ws=wsh)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uh, _, sth = F.solve(pbh, xh, ws=wsh)
            torch.cuda.synchronize()
            sech = time.perf_counter() - t0
            uh = uh.cpu().numpy()
            hj[f"N{Nh}"] = {"value": round(64 / sech, 2), "unit": "points/s", "ms_per_step": round(sech * 1e3, 2),
                            "u_mean": round(float(uh.mean()), 6), "u_sd": round(float(uh.std()), 6),
                            "u_exact": 1.0, "rel_err_vs_exact": round(abs(float(uh.mean()) - 1.0), 5),
                            "status_nonzero_points": int((sth != 0).sum().item()),
                            "paper_cpu_s_per_point_context": 185.06 if Nh == 1000 else 3016.35}
            log(f"[bench] HJ-type d=500 M=100 N={Nh} P=64 (FP64): {sech * 1e3:.1f} ms, u = {uh.mean():.5f} "
                f"(exact 1)")
            del wsh, xh
        small["hj_type_d500_M100_T0.5_P64_fp64"] = hj
        # Allen-Cahn Case 2 (log potential, theta = 0.8 < theta_c = 1.6, manufactured solution
        # 0.25 cos(prod x) e^(cos t - |x|^2)) at the paper's T = 1 and evaluation points x = 0 and (0.1, ..., 0.1):
        # d = 100 at dt = 0.002 / 2^4 (N = 8000) and d = 1000 at dt = 0.0005 / 2^2 (N = 8000), M = 100, FP64
        c2 = {}
        for dc, xv in ((100, 0.0), (100, 0.1), (1000, 0.0)):
            pbc = F.Problem(d=dc, M=100, N=8000, T=1.0, f_kind=F.F_LOG_POT, fp=(0.8, 1.6, 0.25, 0), g_kind=F.G_CASE2,
                            gp=(1.0, 0.25, 0, 0), seed=0, instance=8)
            xc = torch.full((64, dc), xv, dtype=torch.float64, device=dev)
            wsc = F.workspace(pbc, 64, device=dev)
            F.solve(pbc, xc, ws=wsc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uc, _, stc = F.solve(pbc, xc, ws=wsc)
            torch.cuda.synchronize()
            secc = time.perf_counter() - t0
            uc = uc.cpu().numpy()
            exact = 0.25 * math.cos(xv ** dc) * math.exp(1.0 - dc * xv * xv)
            c2[f"d{dc}_x{xv}"] = {"value": round(64 / secc, 2), "unit": "points/s", "ms_per_step": round(secc * 1e3, 2),
                                  "u_mean": round(float(uc.mean()), 6), "u_sd": round(float(uc.std()), 6),
                                  "u_exact": round(exact, 6),
                                  "rel_err_vs_exact": round(abs(float(uc.mean()) - exact) / exact, 5),
                                  "status_nonzero_points": int((stc != 0).sum().item())}
            log(f"[bench] Case 2 d={dc} x={xv} M=100 N=8000 P=64 (FP64): {secc * 1e3:.1f} ms, u = {uc.mean():.5f} "
                f"(exact {exact:.5f})")
            del wsc, xc
        small["allen_cahn_case2_M100_N8000_T1_P64_fp64"] = c2
        # scheme R under x-dependent coefficients mu = 0.05 x - 0.1, sigma = diag(0.2 x + 0.4) (Euler-Maruyama
        # particles, per-point bandwidth and ridge from the moment recursion) at the headline shape
        pbk = F.Problem(d=1000, M=4096, N=20, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC,
                        gp=(0.4, 0, 0, 0), prec=F.F32C, seed=0, instance=0)
        xk = torch.full((1024, 1000), 0.03, dtype=torch.float64, device=dev)
        wsk = torch.empty(F.coef_workspace_size(pbk, 1024, 0.05, 0.2, -0.1, 0.4, tape=True), dtype=torch.uint8,
                          device=dev)
        F.solve_coef(pbk, xk, 0.05, 0.2, -0.1, 0.4, ws=wsk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uk, _, stk = F.solve_coef(pbk, xk, 0.05, 0.2, -0.1, 0.4, ws=wsk)
        torch.cuda.synchronize()
        seck = time.perf_counter() - t0
        itk = F.solve_coef(pbk, xk, 0.05, 0.2, -0.1, 0.4, ws=wsk, return_iters=True)[3]
        # forward with the tape + reverse mode (the design, weights and ridge depend on x0 here)
        ubk = torch.ones(1024, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.solve_coef(pbk, xk, 0.05, 0.2, -0.1, 0.4, ws=wsk, tape=True)
        xbk, _, _, stbk = F.solve_coef_backward(pbk, xk, ubk, wsk, 0.05, 0.2, -0.1, 0.4)
        torch.cuda.synchronize()
        secka = time.perf_counter() - t0
        small["allen_cahn_coef_affine_diag_d1000_P1024_M4096_N20_fp32c"] = {
            "value": round(1024 / seck, 2), "unit": "points/s", "ms_per_step": round(seck * 1e3, 2),
            "coef": {"mu0": 0.05, "sigma0": 0.2, "mu1": -0.1, "sigma1": 0.4}, "cg_iters_per_level": itk,
            "u_mean": round(float(uk.mean().item()), 6), "status_nonzero_points": int((stk != 0).sum().item()),
            "fwd_adj": {"value": round(1024 / secka, 2), "unit": "points/s", "ms_per_step": round(secka * 1e3, 2),
                        "workspace_with_tape_GiB": round(wsk.numel() / 2 ** 30, 2),
                        "status_nonzero_points": int((stbk != 0).sum().item())}}
        log(f"[bench] x-dependent coefficients d=1000 M=4096 P=1024 N=20 (FP32C): {seck * 1e3:.1f} ms, "
            f"forward + adjoint {secka * 1e3:.1f} ms")
        del xbk
        del wsk, xk

    # ---------------- paper-literal per-anchor scheme at the paper's Burgers runtime setting:
    # d = 10^4, M = 100, dt = 0.003 (N = 100), T = 0.3, x0 = 0, as 64 independent replicas of the point
    literal = None
    if not args.no_literal:
        dl, Ml, Nl, Pl, Tl = 10000, 100, 100, 64, 0.3
        sl = math.sqrt(2.0)
        gvl = torch.full((dl,), 1.0 / dl, dtype=torch.float64, device=dev)
        pbl = F.Problem(d=dl, M=Ml, N=Nl, T=Tl, s=sl, f_kind=F.F_BURGERS, fp=(sl / dl, dl / (sl * sl) + 0.5, 0, 0),
                        g_kind=F.G_LOGISTIC, gp=(Tl, 0, 0, 0), gvec=gvl, eps_h=1.0, ridge_rel=1e-3, instance=6)
        xl = torch.zeros((Pl, dl), dtype=torch.float64, device=dev)
        torch.cuda.empty_cache()
        # a workspace that keeps every level's particles (52 GB): no reversal by regenerated increments
        wsl = torch.empty(F.literal_workspace_size(pbl, Pl, stored=True), dtype=torch.uint8, device=dev)
        F.solve_literal(pbl, xl, ws=wsl)
        torch.cuda.synchronize()
        F.launch_timer(True)
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps)):
            ul, stl, _, _ = F.solve_literal(pbl, xl, ws=wsl)
        torch.cuda.synchronize()
        secl = (time.perf_counter() - t0) / max(1, args.steps)
        F.launch_timer(False)
        ms_l, work_l = F.launch_timer_read(with_bytes=True)
        kinds_l = F.launch_timer_kinds()
        legs = {}
        for name, kind in (("gram", F.TIMED_LITERAL_GRAM), ("anchors", F.TIMED_LITERAL_ANCHORS)):
            sel = kinds_l == kind
            t_ms = float(ms_l[sel].mean())
            tf = float(work_l[sel][0]) / (t_ms * 1e-3) / 1e12
            legs[name] = {"launches": int(sel.sum()), "avg_ms": round(t_ms, 4),
                          "share_of_solve": round(float(ms_l[sel].sum()) / 1e3 / (secl * max(1, args.steps)), 3),
                          "flops_per_launch": float(work_l[sel][0]), "achieved_TFLOPs": round(tf, 2),
                          "frac_of_fp64_peak": round(tf / FP64_PEAK_TFLOPS, 4)}
        ul = ul.cpu().numpy()
        literal = {"value": round(Pl / secl, 3), "unit": "points/s", "ms_per_step": round(secl * 1e3, 3),
                   "dtype": "f64", "config": {"workload": "literal_burgers_d10000_M100_N100_T0.3_P64", "d": dl,
                                              "M": Ml, "N": Nl, "T": Tl, "points": Pl, "x0": "0 (replicas)",
                                              "ridge_rel": 1e-3, "kernel_h": 1.0},
                   "stored_path_GB": round(wsl.numel() / 1e9, 2),
                   "u_mean": round(float(ul.mean()), 6), "u_sd": round(float(ul.std()), 6), "u_exact": 0.5,
                   "status_nonzero_points": int((stl != 0).sum().item()), "kernels": legs,
                   "paper_cpu_s_per_point_context": 1040.15}
        log(f"[bench] literal per-anchor d=1e4 M=100 N=100 P=64: {secl * 1e3:.1f} ms "
            f"(gram {legs['gram']['avg_ms']:.3f} ms/level, anchors {legs['anchors']['avg_ms']:.3f} ms/level)")
        del wsl
        # the paper's second particle count at this setting, M = 200 (eight-wavefront anchor layout), with the
        # minimal workspace (the path reversed by regenerated increments)
        pb2 = F.Problem(d=dl, M=200, N=Nl, T=Tl, s=sl, f_kind=F.F_BURGERS, fp=(sl / dl, dl / (sl * sl) + 0.5, 0, 0),
                        g_kind=F.G_LOGISTIC, gp=(Tl, 0, 0, 0), gvec=gvl, eps_h=1.0, ridge_rel=1e-3, instance=6)
        ws2 = torch.empty(F.literal_workspace_size(pb2, Pl), dtype=torch.uint8, device=dev)
        F.solve_literal(pb2, xl, ws=ws2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u2, st2, _, _ = F.solve_literal(pb2, xl, ws=ws2)
        torch.cuda.synchronize()
        sec2 = time.perf_counter() - t0
        if not args.no_cpu_baseline:
            # the oracle on a bounded sample: one point, 6 of the 100 levels (same d, M, dt), scaled by 100 / 6
            from oracle import literal as OL
            from oracle import scheme as OS
            ocw = dict(d=dl, M=Ml, N=6, T=0.003 * 6, s=sl, f_kind=OS.F_BURGERS, fp=(sl / dl, dl / (sl * sl) + 0.5, 0, 0),
                       g_kind=OS.G_LOGISTIC, gp=(Tl, 0, 0, 0), gvec=np.full(dl, 1.0 / dl), ridge_rel=1e-3, eps_h=1.0,
                       instance=6)
            t0 = time.perf_counter()
            OL.solve_point(OS.Problem(**ocw), np.zeros(dl), 0)
            sec_o = (time.perf_counter() - t0) * Nl / 6
            literal["cpu_oracle"] = {"value": round(1.0 / sec_o, 5), "unit": "points/s", "kind": "oracle",
                                     "cores": int(threads),
                                     "sample": "1 point, 6 of the 100 levels (same d, M, dt), time scaled by 100/6"}
            log(f"[bench] literal oracle sample: {sec_o:.1f} s per point (scaled)")
        literal["M200"] = {"value": round(Pl / sec2, 3), "unit": "points/s", "ms_per_step": round(sec2 * 1e3, 3),
                           "u_mean": round(float(u2.mean().item()), 6),
                           "status_nonzero_points": int((st2 != 0).sum().item()),
                           "paper_cpu_s_per_point_context": 2189.28}
        log(f"[bench] literal per-anchor d=1e4 M=200 N=100 P=64: {sec2 * 1e3:.1f} ms")
        del ws2, xl
        # the shape of the paper's HJ-type runtime table (d = 500, dt = 0.0005, T = 0.5: N = 1000 levels), with
        # the HJB family f = -|z|^2, g = ln((1 + |x|^2) / 2) standing in for its equation; stored path
        torch.cuda.empty_cache()
        hj = {}
        for Mh in (50, 100):
            pbh = F.Problem(d=500, M=Mh, N=1000, T=0.5, f_kind=F.F_HJB, fp=(1.0, 0, 0, 0), g_kind=F.G_HJB_LOG,
                            gp=(1.0, 0, 0, 0), eps_h=1.0, ridge_rel=1e-3, instance=9)
            xh = torch.zeros((Pl, 500), dtype=torch.float64, device=dev)
            wsh = torch.empty(F.literal_workspace_size(pbh, Pl, stored=True), dtype=torch.uint8, device=dev)
            F.solve_literal(pbh, xh, ws=wsh)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uh, sth, _, _ = F.solve_literal(pbh, xh, ws=wsh)
            torch.cuda.synchronize()
            sech = time.perf_counter() - t0
            hj[f"M{Mh}"] = {"value": round(Pl / sech, 3), "unit": "points/s", "ms_per_step": round(sech * 1e3, 3),
                            "status_nonzero_points": int((sth != 0).sum().item()),
                            "paper_cpu_s_per_point_context": 89.07 if Mh == 50 else 185.06}
            log(f"[bench] literal HJB-type d=500 M={Mh} N=1000 P=64: {sech * 1e3:.1f} ms")
            del wsh, xh
        literal["hj_shape_d500_N1000"] = hj
        # x-dependent coefficients: geometric family mu = mu0 x, sigma = sigma0 diag(x), the path stored per level
        dg_, Mg, Ng, Pg = 1000, 100, 50, 64
        pbg = F.Problem(d=dg_, M=Mg, N=Ng, T=0.5, f_kind=F.F_HJB, fp=(1.0, 0, 0, 0), g_kind=F.G_HJB_LOG,
                        gp=(1.0, 0, 0, 0), eps_h=1.0, ridge_rel=1e-3, instance=7)
        xg = torch.ones((Pg, dg_), dtype=torch.float64, device=dev)
        wsg = torch.empty(F.literal_coef_workspace_size(pbg, Pg, 0.05, 0.2), dtype=torch.uint8, device=dev)
        F.solve_literal_geometric(pbg, xg, 0.05, 0.2, ws=wsg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps)):
            ug, stg, _, _ = F.solve_literal_geometric(pbg, xg, 0.05, 0.2, ws=wsg)
        torch.cuda.synchronize()
        secg = (time.perf_counter() - t0) / max(1, args.steps)
        literal["geometric_coefficients"] = {
            "value": round(Pg / secg, 3), "unit": "points/s", "ms_per_step": round(secg * 1e3, 3),
            "config": {"workload": "literal_geometric_hjb_d1000_M100_N50_P64", "mu0": 0.05, "sigma0": 0.2,
                       "x0": "1 (replicas)", "stored_path_GB": round(wsg.numel() / 1e9, 2)},
            "u_mean": round(float(ug.mean().item()), 6), "status_nonzero_points": int((stg != 0).sum().item())}
        log(f"[bench] literal geometric d=1e3 M=100 N=50 P=64: {secg * 1e3:.1f} ms")
        del wsg, xg

    # ---------------- shared increments: d = 10^4, 4096 points, M = 2048, N = 20 on the matrix cores
    shared = None
    if not args.no_shared:
        Ps, ds, Ms = 4096, 10000, 2048
        pbs = F.Problem(d=ds, M=Ms, N=20, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0.0, 0.0), g_kind=F.G_AC,
                        gp=(0.4, 0.0, 0.0, 0.0), shared_dw=1, prec=F.F32C, seed=0, instance=4)
        xs_np = workloads.points("normal_over_sqrt_d", Ps, ds, seed=7)
        xs = torch.tensor(xs_np, dtype=torch.float64, device=dev)
        wss = F.workspace(pbs, Ps, device=dev)
        sec_s, us_, gs_, sts_, _ = timed_solves(F, torch, pbs, xs, wss, 1, max(1, args.steps))
        log(f"[bench] shared fp32c d=1e4 P=4096 M=2048: {sec_s * 1e3:.1f} ms/solve")
        del wss
        torch.cuda.empty_cache()
        # the dominant GEMM of that leg, timed live on torch's stream (the library launches there)
        ldp = F.state_ld(pbs)
        A = torch.randn((Ps, ldp), dtype=torch.float32, device=dev)
        B = torch.randn((Ms, ldp), dtype=torch.float32, device=dev)
        C = torch.empty((Ps, Ms), dtype=torch.float32, device=dev)
        F.gemm(A, B, nt=True, C=C)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            F.gemm(A, B, nt=True, C=C)
        e1.record()
        torch.cuda.synchronize()
        gemm_ms = e0.elapsed_time(e1) / 5
        tflops = 2.0 * Ps * Ms * ldp / (gemm_ms * 1e-3) / 1e12
        del A, B, C
        torch.cuda.empty_cache()
        # forward with the tape + reverse mode of L = sum_p u_p (the C4 training-style step)
        wsst = F.workspace(pbs, Ps, tape=True, device=dev)
        ubs = torch.ones(Ps, dtype=torch.float64, device=dev)
        F.solve(pbs, xs, tape=True, ws=wsst)
        F.solve_backward(pbs, xs, ubs, wsst)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nfa = max(1, args.steps)
        for _ in range(nfa):
            F.solve(pbs, xs, tape=True, ws=wsst)
            _, _, _, st_sa = F.solve_backward(pbs, xs, ubs, wsst)
        torch.cuda.synchronize()
        sec_sfa = (time.perf_counter() - t0) / nfa
        log(f"[bench] shared fp32c fwd+adj: {sec_sfa * 1e3:.1f} ms")
        tape_gib = wsst.numel() / 2**30
        del wsst
        torch.cuda.empty_cache()
        shared = {"value": round(Ps / sec_s, 2), "unit": "points/s", "ms_per_step": round(sec_s * 1e3, 3),
                  "fwd_adj": {"value": round(Ps / sec_sfa, 2), "unit": "points/s", "ms_per_step": round(sec_sfa * 1e3, 3),
                              "workspace_with_tape_GiB": round(tape_gib, 2),
                              "status_nonzero_points": int((st_sa != 0).sum().item())},
                  "dtype": "fp32c (FP32 MFMA, FP64 Newton)",
                  "config": {"workload": "shared_allen_cahn_d10000_P4096_M2048_N20", "shared_increments": True},
                  "roofline": {"bound": "mfma", "kernel": "k_gemm_f32p<NT, FP64-folded> [P x ld] x [M x ld]^T",
                               "achieved": round(tflops, 2), "peak": 157.3, "unit": "TFLOP/s",
                               "frac": round(tflops / 157.3, 4), "avg_launch_ms": round(gemm_ms, 4),
                               "flops_per_launch": 2 * Ps * Ms * ldp},
                  "status_nonzero_points": int((sts_ != 0).sum().item())}
        del xs
        torch.cuda.empty_cache()

    # ---------------- batched: 64 uneven HJB instances (the 256-point workload cut to --batched-points per
    # instance so the leg stays within a minute), tiled schedule
    batched = None
    if not args.no_batched:
        insts = workloads.batched_instances(64)
        Pb = args.batched_points
        probs, xb = [], []
        for it in insts:
            probs.append(F.Problem(d=it["d"], M=it["M"], N=20, T=1.0, f_kind=F.F_HJB, fp=(it["lam"], 0, 0, 0),
                                   g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0), prec=F.F32C, seed=0, instance=it["instance"]))
            xb.append(torch.tensor(workloads.points("uniform", Pb, it["d"], seed=100 + it["instance"]),
                                   dtype=torch.float64, device=dev))
        # one small warm-up batch (thread pool, streams, first launches), then the timed batch
        F.solve_batched(probs[:2], [x[:1] for x in xb[:2]])
        wsb = F.batched_workspace(probs, xb)
        torch.cuda.synchronize()
        F.launch_timer(True)
        t0 = time.perf_counter()
        ub, gb, stb = F.solve_batched(probs, xb, ws=wsb)
        torch.cuda.synchronize()
        sec_b = time.perf_counter() - t0
        F.launch_timer(False)
        loop_ms_b = float(F.launch_timer_read()[F.launch_timer_kinds() == F.TIMED_CG_LOOP].sum())
        bytes_b = F.batched_cg_bytes(probs, xb, wsb)
        del wsb
        log(f"[bench] batched 64 instances x {Pb} points (tiled): {sec_b * 1e3:.1f} ms, CG products "
            f"{bytes_b / sec_b / 1e9:.0f} GB/s over the wall time")
        ubs = [torch.ones(x.shape[0], dtype=torch.float64, device=dev) for x in xb]
        wsba = F.batched_workspace(probs, xb, adjoint=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rb = F.solve_batched_backward(probs, xb, ubs, ws=wsba)
        torch.cuda.synchronize()
        sec_ba = time.perf_counter() - t0
        bytes_ba = F.batched_cg_bytes(probs, xb, wsba, adjoint=True)
        del wsba
        log(f"[bench] batched 64 instances x {Pb} points fwd+adj (tiled): {sec_ba * 1e3:.1f} ms")
        n_pts = Pb * len(insts)
        elems = sum(Pb * it["M"] * it["d"] for it in insts)
        def traffic(nbytes, sec):
            return {"bytes": nbytes, "achieved_GBs": round(nbytes / sec / 1e9, 1),
                    "frac_of_hbm_peak": round(nbytes / sec / 1e9 / HBM_PEAK_GBS, 4)}

        batched = {"value": round(n_pts / sec_b, 2), "unit": "points/s", "ms_per_step": round(sec_b * 1e3, 3),
                   "dtype": "fp32c", "schedule": "tiled: (instance, point-tile) items over 3 streams, each level's "
                                                 "CG one device-side loop launch",
                   "fwd_adj": {"value": round(n_pts / sec_ba, 2), "unit": "points/s",
                               "ms_per_step": round(sec_ba * 1e3, 3),
                               "cg_product_traffic": traffic(bytes_ba, sec_ba),
                               "status_nonzero_points": int(sum(int((s_ != 0).sum().item()) for s_ in rb[4]))},
                   "config": {"workload": "batched_hjb_64_instances", "points_per_instance": Pb,
                              "d": "uniform over {100, 500, 1000, 5000, 10000}", "M": "multiples of 64 in [512, 8192]",
                              "T": 1.0, "N": 20, "f": "-lam |z|^2, lam ~ U[0.5, 2]", "g": "ln((1+|x|^2)/2)",
                              "x0": "U[-1,1]^d", "state_elements": elems},
                   "cg_product_traffic": dict(traffic(bytes_b, sec_b),
                                              loop_stream_time_share=round(loop_ms_b / 1e3 / (3 * sec_b), 3),
                                              note="bytes: rows streamed by every CG product (device count) x d x 4 "
                                                   "B, over the wall time of the whole batched call"),
                   "status_nonzero_points": int(sum(int((s_ != 0).sum().item()) for s_ in stb))}
        del rb, ubs
        del xb, ub, gb, stb
        torch.cuda.empty_cache()

    # ---------------- the batched workload at its configured size: 64 instances x 256 points, forward, run
    # as eight calls of eight instances each (each call prints when it ends)
    batched_full = None
    if args.batched_full_forward:
        insts = workloads.batched_instances(64)
        Pf = 256
        tot_s, tot_b, nz = 0.0, 0.0, 0
        for s0 in range(0, len(insts), 8):
            sl = insts[s0:s0 + 8]
            probs = [F.Problem(d=it["d"], M=it["M"], N=20, T=1.0, f_kind=F.F_HJB, fp=(it["lam"], 0, 0, 0),
                               g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0), prec=F.F32C, seed=0, instance=it["instance"])
                     for it in sl]
            xs = [torch.tensor(workloads.points("uniform", Pf, it["d"], seed=100 + it["instance"]),
                               dtype=torch.float64, device=dev) for it in sl]
            wsf = F.batched_workspace(probs, xs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uf, _, stf = F.solve_batched(probs, xs, want_grad=False, ws=wsf)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            nb = F.batched_cg_bytes(probs, xs, wsf)
            tot_s += sec
            tot_b += nb
            nz += int(sum(int((q != 0).sum().item()) for q in stf))
            log(f"[bench] full batched slice {s0 // 8 + 1}/8 (instances {s0}..{s0 + len(sl) - 1}, d "
                f"{sorted(set(it['d'] for it in sl))}): {sec:.1f} s, CG products {nb / sec / 1e12:.2f} TB/s")
            del wsf, xs, uf, stf
            torch.cuda.empty_cache()
        batched_full = {"value": round(Pf * len(insts) / tot_s, 2), "unit": "points/s", "seconds": round(tot_s, 2),
                        "config": {"workload": "batched_hjb_64_instances", "points_per_instance": Pf,
                                   "calls": "8 calls of 8 instances"},
                        "cg_product_traffic": {"bytes": tot_b, "achieved_GBs": round(tot_b / tot_s / 1e9, 1),
                                               "frac_of_hbm_peak": round(tot_b / tot_s / 1e9 / HBM_PEAK_GBS, 4)},
                        "status_nonzero_points": nz}
        log(f"[bench] full batched 64 x 256 forward: {tot_s:.1f} s, {Pf * len(insts) / tot_s:.1f} points/s, CG "
            f"products {tot_b / tot_s / 1e12:.2f} TB/s")

    value = P / sec32
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec32 * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32c", "data": "synthetic",
        "config": {"workload": "allen_cahn_d1000_P1024_M4096_N20", "d": 1000, "points": P, "M": 4096, "N": 20,
                   "T": 0.3, "f": "u-u^3", "g": "1/(2+0.4|x|^2)", "x0": "N(0,0.25 I)", "kernel_h": 1.0,
                   "ridge_rel": 1e-3, "cg_rtol": 1e-7},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": None if sec64 is None else {"value": round(P / sec64, 3), "unit": "points/s",
                                             "ms_per_step": round(sec64 * 1e3, 3), "cg_rtol": 1e-13,
                                             "cg_iters_per_level": it64},
        "fp64_equal_tolerance": None if sec64e is None else {
            "value": round(P / sec64e, 3), "unit": "points/s", "ms_per_step": round(sec64e * 1e3, 3),
            "cg_rtol": 1e-7, "cg_iters_per_level": it64e},
        "fwd_adj": {"value": round(P / sec_fa, 3), "unit": "points/s", "ms_per_step": round(sec_fa * 1e3, 3),
                    "dtype": "fp32c", "loss": "sum_p u(0, x0_p)", "outputs": "d/dx0 [P][d], d/dgp, d/dfp"},
        # FP32C and FP64 at the same CG tolerance (1e-7): the speedup at equal accuracy; the FP64 leg at
        # 1e-13 also runs more CG iterations, so its ratio mixes precision and tolerance
        "speedup_fp32c_over_fp64_equal_tolerance": None if sec64e is None else round(sec64e / sec32, 3),
        "speedup_fp32c_over_fp64_mixed_tolerance": None if sec64 is None else round(sec64 / sec32, 3),
        "rel_err_vs_fp64_oracle": errs or None,
        "cg_iters_per_level_fp32c": it32,
        "adjoint_cg_iters_per_level_fp32c": it_adj,
        "whole_job_state_traffic": whole_job,
        "other_configurations": small,
        "shared_increments_mfma": shared,
        "literal_per_anchor": literal,
        "batched": batched,
        "batched_full_forward": batched_full,
        "reverse_sweep_avg_ms_fp32c": round(rev32_ms, 4),
        "status_nonzero_points": int(np.count_nonzero(st32)),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
