#!/usr/bin/env python
"""Benchmark of the geometric alpha-SA multigrid hot path on one MI355X.

Workload: 2D Poisson, SIPG p=3 (10 dofs per triangle) on the Delaunay
triangulation of 256^2 seeded jittered points (130,050 triangles, 1,300,500
dofs), 5-level hierarchy by recursive coordinate bisection, 3 adaptive
candidates, V(3,3) block Jacobi with adaptive damping; right-hand side(s)
N(0,1) from seed 1.  The hierarchy is built once (setup time reported
separately); a step is one solve of the batch of right-hand sides to a true
relative residual of 1e-8 from x = 0, with the V-cycle as preconditioner:

* mixed : FP32 V-cycle inside FP64 flexible CG (the reported value),
* fp64  : FP64 V-cycle inside FP64 CG (reported beside it).

Prints one JSON line: metric, value (solves/s, from the median of the timed
solves), timing, roofline of the dominant kernel, the forward error of both
paths against a reference independent of the GPU, CPU baseline and the
per-path details.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def level_bytes(info, w, m, nu):
    """Algorithmic bytes of one V(nu,nu) visit of a non-coarsest level: one pass
    over D_k^{-1} (the first sweep, which also forms c = D^{-1} b), 2nu passes over
    S_k = D_k^{-1} A_k (2nu - 1 sweeps and the residual), one over T_k and R_k D_k,
    and (6nu+6) passes over level-k vectors.  A level that restricts through
    M_k = R_k (D_k - omega A_k) has no residual pass: 2nu - 1 passes over S_k, one
    over T_k and M_k, and (6nu+4) vector passes (the last pre-sweep writes its
    residual, which M_k reads)."""
    nS = info.nnzb_S or info.nnzb  # D^-1 A as stored: its off-diagonal blocks
    S = nS * info.nb * info.nb * w + 4 * nS + 4 * (info.n_units + 1)
    D = info.n_units * info.nb * info.nb * w
    TR = info.nnzb_T * info.nb * info.s * w + 4 * info.nnzb_T + 4 * (info.n_units + 1)
    # (on the 16-column tiles the library restricts through M only on levels of 2,048 or more coarse block rows)
    if getattr(info, "restrict_resid", 0) and not (m % 16 == 0 and info.n_agg < 2048):
        MM = info.nnzb_M * info.nb * info.s * w + 4 * info.nnzb_M + 4 * (info.n_agg + 1)
        return (2 * nu - 1) * S + D + (6 * nu + 4) * info.n * m * w + TR + MM
    RR = info.nnzb_T * info.nb * info.s * w + 4 * info.nnzb_T + 4 * (info.n_agg + 1)
    return 2 * nu * S + D + (6 * nu + 6) * info.n * m * w + TR + RR


def sweep_bytes(info, w, m):
    """Algorithmic bytes of one block-Jacobi sweep as the V-cycle runs it,
    y = x + omega (c - S x) with S = D^-1 A and c = D^-1 b: S's off-diagonal
    blocks (values and indices; its diagonal blocks are the identity), x and c
    read once, y written once."""
    nS = info.nnzb_S or info.nnzb
    return (nS * info.nb * info.nb * w + 4 * nS + 4 * (info.n_units + 1)
            + 3 * info.n * m * w)


def sliced_kernels_sha256():
    """sha256 of the device code of the sliced-layout kernels (sell_row,
    k_sweep, k_spmv: the level-0 sweep the counters measure), up to their
    host-side launchers."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2504_13373_amd", "csrc", "kernels.hip")).read()
    a = src.index("// ============================================================ BSR kernels")
    b = src.index("template <typename T, int M, bool CHUNKED = false>\nstatic hipError_t sweep_m")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def measured_traffic(kernel):
    """L2-miss bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current sliced kernels (else None)."""
    f = os.path.join(ROOT, "profiles", "sweep_level0_poisson2d_p3_256_traffic.txt")
    if not os.path.exists(f):
        return None
    head, rows = {}, {}
    for line in open(f):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("kernel="):
            kv = dict(x.split("=", 1) for x in line.split(";"))
            rows[kv["kernel"]] = float(kv["hbm_bytes"])
        elif "=" in line:
            k, v = line.split("=", 1)
            head[k] = v
    if head.get("sliced_kernels_sha256") != sliced_kernels_sha256():
        return None
    return rows.get(kernel)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rhs", type=int, default=1, help="right-hand sides per solve")
    ap.add_argument("--workload", choices=["poisson2d", "convdiff", "poisson3d", "serving", "hex"],
                    default="poisson2d",
                    help="poisson2d: the headline workload; convdiff: LDG convection-diffusion Peclet sweep "
                         "with FGMRES(30); poisson3d: 3D tetrahedra, 16 right-hand sides; serving: a Poisson "
                         "stream of solve requests over a catalogue of operators; hex: the structured "
                         "hexahedral Poisson problem (Q1, IP and LDG, 2^M cubes per direction, M = 3, 4, 5)")
    ap.add_argument("--catalogue", type=int, default=32, help="serving: operator instances")
    ap.add_argument("--t-max", type=float, default=2e5, help="serving: largest triangle count")
    ap.add_argument("--serve-duration", type=float, default=60.0, help="serving: seconds of arrivals counted")
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="serving: seconds of arrivals not counted")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: HBM budget of the request state")
    ap.add_argument("--side", type=int, default=None,
                    help="grid points per side (2D; defaults 256 / 363) or cells per side (3D; default 64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="also run a plain elementwise copy of MB megabytes (reads and writes MB each), "
                         "the reference for the HBM traffic counters")
    ap.add_argument("--serve", type=int, default=16, metavar="N",
                    help="requests of the serving run (0: skip it)")
    ap.add_argument("--serve-width", type=int, default=4, help="right-hand sides per server batch")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate in requests/s (0: all requests arrive at once)")
    ap.add_argument("--skip-fp64", action="store_true", help="poisson3d: time the mixed path only")
    ap.add_argument("--hex-m", type=int, nargs="*", default=[3, 4, 5], help="hex: refinement levels M")
    ap.add_argument("--hex-r", type=int, nargs="*", default=[16, 64], help="hex: candidate counts r (64: the median dofs of a level-1 aggregate, the paper's own choice)")
    ap.add_argument("--hex-flux", nargs="*", default=["ip", "ldg"], help="hex: fluxes (ip, ldg)")
    ap.add_argument("--hex-p", type=int, nargs="*", default=[1], help="hex: polynomial degrees (Q_p)")
    ap.add_argument("--hex-hstar", action="store_true", help="hex: also the h*-hierarchy for p >= 2")
    ap.add_argument("--hex-matfree", type=int, nargs="*", default=[0],
                    help="hex: matrix-free levels kappa (levels 1..kappa keep no A_k)")
    ap.add_argument("--mixed-outer", choices=["fcg", "fgmres"], default="fcg",
                    help="poisson2d: outer iteration of the mixed path: flexible CG with residual replacement, or "
                         "restarted FGMRES from the true FP64 residual (iterative refinement)")
    ap.add_argument("--restart", type=int, default=30, help="FGMRES restart length")
    ap.add_argument("--oversample", action="store_true",
                    help="poisson2d: also the paper's oversampled setup (r = the median dofs of a level-1 "
                         "aggregate, s_J per aggregate, levels until the coarsest holds at most 2,048 dofs)")
    ap.add_argument("--no-restrict-resid", action="store_true",
                    help="form each level's residual and restrict it through R D instead of through M = R (D - omega A)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (no amgdg_autotune before timing)")
    ap.add_argument("--tune-lanes", action="store_true",
                    help="let the autotuner also pick the block-CSR lane widths (changes rounding)")
    ap.add_argument("--max-it", type=int, default=50000,
                    help="iteration cap per solve (profiling runs cap it; the reported value needs convergence)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2504_13373_amd as am
    from workloads import configs

    dev = torch.device("cuda:0")
    if args.workload == "convdiff":
        return bench_convdiff(args, am, torch, dev)
    if args.workload == "poisson3d":
        return bench_poisson3d(args, am, torch, dev)
    if args.workload == "serving":
        return bench_serving_stream(args, am, torch, dev)
    if args.workload == "hex":
        return bench_hex(args, am, torch, dev)
    args.side = args.side or 256
    log(f"generating workload (side {args.side})")
    t0 = time.perf_counter()
    w = configs.poisson2d_delaunay(side=args.side, n_rhs=args.rhs)
    log(f"workload: {w.mesh.n_elem} elements, {w.A.n} dofs, {w.A.nnzb} blocks ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h, agg = am.setup_from_workload(w, mixed=True, restrict_resid=int(not args.no_restrict_resid))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    infos = [am.amgdg_level_info_get(h, k) for k in range(h.n_levels)]
    log(f"setup {setup_s:.2f} s; levels n = {[i.n for i in infos]}, omega = {[round(i.omega, 4) for i in infos[:-1]]}")

    m = args.rhs
    tuning = _autotune(args, am, torch, h, m)
    b = torch.as_tensor(w.b.reshape(w.A.n, m) if m > 1 else w.b).to(dev).contiguous()
    x = torch.zeros_like(b)
    maxit = args.max_it

    def solve(method, prec):
        x.zero_()
        rc, st = am.amgdg_solve(h, b, x, method, prec, 1e-8, maxit, restart=args.restart)
        return rc, st

    mixed_outer = am.AMGDG_FGMRES if args.mixed_outer == "fgmres" else am.AMGDG_FCG
    paths = {"mixed": (mixed_outer, am.AMGDG_MIXED), "fp64": (am.AMGDG_PCG, am.AMGDG_FP64)}
    res = {}
    A = w.A.to_scipy()
    bh = w.b.reshape(w.A.n, m) if m > 1 else w.b[:, None]
    for name, (meth, prec) in paths.items():
        for i in range(args.warmup):
            rc, st = solve(meth, prec)
            log(f"warmup {name} {i}: rc {rc}, iterations {st.max_iterations}")
        torch.cuda.synchronize()
        times = []
        for i in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = solve(meth, prec)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            log(f"step {name} {i}: {times[-1] * 1e3:.1f} ms, iterations {st.max_iterations}, rc {rc}")
        xh = x.cpu().numpy().reshape(w.A.n, m)
        true_rel = float(np.max(np.linalg.norm(bh - A @ xh, axis=0) / np.linalg.norm(bh, axis=0)))
        res[name] = dict(times=times, its=st.max_iterations, rc=rc, true_rel=true_rel, x=xh)
    # forward error against a reference that does not come from the GPU: a
    # manufactured problem b* = A x* (x* ~ N(0,1), seed 5, b* formed in FP64 on
    # the host) solved untimed by both paths; and the two paths' solutions of
    # the timed right-hand side against each other
    xstar = np.random.default_rng(5).standard_normal((w.A.n, m))
    bstar = torch.as_tensor(np.ascontiguousarray((A @ xstar).reshape(b.shape))).to(dev)
    for name, (meth, prec) in paths.items():
        xs = torch.zeros_like(bstar)
        rc, st = am.amgdg_solve(h, bstar, xs, meth, prec, 1e-8, maxit)
        xsh = xs.cpu().numpy().reshape(w.A.n, m)
        res[name]["fwd_err"] = float(np.max(np.linalg.norm(xsh - xstar, axis=0) / np.linalg.norm(xstar, axis=0)))
        log(f"{name}: forward error vs the manufactured solution {res[name]['fwd_err']:.3e} ({st.max_iterations} it)")
    mix_vs_64 = float(np.max(np.linalg.norm(res["mixed"]["x"] - res["fp64"]["x"], axis=0)
                             / np.linalg.norm(res["fp64"]["x"], axis=0)))

    # V-cycle HBM rate (algorithmic bytes / measured time), both precisions
    nu = w.params.t_pre
    stream = torch.cuda.current_stream()
    vc = {}
    for name, (prec, wb, dt) in {"fp64": (am.AMGDG_FP64, 8, torch.float64),
                                 "fp32": (am.AMGDG_MIXED, 4, torch.float32)}.items():
        r = torch.randn(w.A.n * m, dtype=dt, device=dev).reshape(b.shape)
        z = torch.zeros_like(r)
        for _ in range(3):
            am.amgdg_vcycle(h, r, z, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            am.amgdg_vcycle(h, r, z, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps * 1e-3
        nN = infos[-1].n
        byts = sum(level_bytes(i, wb, m, nu) for i in infos[:-1]) + nN * nN * 8 + 2 * nN * m * 8
        vc[name] = dict(ms=t * 1e3, gbps=byts / t / 1e9, bytes=byts)
        log(f"V-cycle {name}: {t * 1e3:.3f} ms, {byts / 1e9:.3f} GB algorithmic, {byts / t / 1e9:.0f} GB/s")

    # dominant kernel: the level-0 block-Jacobi sweep in the row-scaled form the
    # V-cycle runs, timed with HIP events on the stream it is launched on (one
    # kernel launch per call with internal ordering)
    kern = {}
    for name, (prec, wb, dt) in {"fp32": (am.AMGDG_MIXED, 4, torch.float32),
                                 "fp64": (am.AMGDG_FP64, 8, torch.float64)}.items():
        xx = torch.randn(w.A.n * m, dtype=dt, device=dev).reshape(b.shape)
        bb = torch.randn_like(xx)
        yy = torch.zeros_like(xx)
        for _ in range(5):
            am.amgdg_apply(h, 0, am.AMGDG_OP_SWEEP_SCALED, xx, bb, yy, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.kernel_reps):
            am.amgdg_apply(h, 0, am.AMGDG_OP_SWEEP_SCALED, xx, bb, yy, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / args.kernel_reps * 1e-3
        byts = sweep_bytes(infos[0], wb, m)
        kern[name] = dict(us=t * 1e6, gbps=byts / t / 1e9, bytes=byts)
        log(f"level-0 sweep {name}: {t * 1e6:.1f} us, {byts / 1e6:.1f} MB, {byts / t / 1e9:.0f} GB/s")
        if name == "fp32":
            t = _evicted_launch_time(torch, dev, stream, lambda: am.amgdg_apply(
                h, 0, am.AMGDG_OP_SWEEP_SCALED, xx, bb, yy, precision=prec, flags=am.AMGDG_INTERNAL_ORDER),
                args.kernel_reps)
            kern["fp32_cold"] = dict(us=t * 1e6, gbps=byts / t / 1e9, bytes=byts)
            log(f"level-0 sweep fp32, cache evicted: {t * 1e6:.1f} us, {byts / t / 1e9:.0f} GB/s")
    copy_gbps = _copy_bandwidth(torch, dev, stream)

    _copy_calibration(args, torch, dev)

    serving = None
    if args.serve > 0:
        serving = serve_bench(am, h, w.A.n, dev, args.serve, args.serve_width, args.serve_rate, maxit)

    oversampled = bench_oversampled(args, am, torch, dev, w, maxit) if args.oversample else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, res["fp64"]["its"])

    mixed_t = float(np.median(res["mixed"]["times"]))
    fp64_t = float(np.median(res["fp64"]["times"]))
    k = kern["fp64"]
    line = {
        "metric": "solves/sec + HBM GB/s of V-cycle to 1e-8 rel. resid; mixed vs FP64, p99 latency",
        "value": m / mixed_t,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed_t * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle + f64 Krylov",
        "data": "synthetic",
        "config": {
            "workload": f"2D Poisson SIPG p=3, Delaunay of {args.side}^2 jittered points "
                        f"({w.mesh.n_elem} triangles, {w.A.n} dofs), 5-level RCB hierarchy, r=3, V(3,3), "
                        f"tol 1e-8, {m} RHS per solve",
            "rhs_per_solve": m,
            "outer": ("flexible CG" if args.mixed_outer == "fcg" else f"FGMRES({args.restart}) iterative refinement")
                     + " (mixed) / CG (fp64)",
            "outer_note": "the mixed path's outer iteration is flexible CG with residual replacement: FGMRES(30) "
                          "iterative refinement around the same FP32 V-cycle stagnates on this workload (30,000 "
                          "iterations, relative residual 7.5e-6; --mixed-outer fgmres)",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "level-0 FP64 block-Jacobi sweep on D^-1 A (k_spmv<double,1,S_SWEEP,false,false>; the "
                      "diagonal blocks of D^-1 A are the identity and are not stored), the kernel with the most "
                      f"GPU time in this run; its {k['bytes'] / 1e6:.0f} MB working set exceeds the 256 MB "
                      "Infinity Cache, so back-to-back launches in one direction find none of it cached (inside "
                      "the V-cycles consecutive passes alternate direction and find part of it cached)",
            "achieved": k["gbps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": k["gbps"] / HBM_PEAK_GBS,
            "traffic": measured_traffic("k_spmv<double, 1, 3, false, false>"),
            "traffic_kind": "L2-miss bytes (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size); the "
                            "memory-side cache or HBM serves them",
            "bytes_per_launch": k["bytes"],
            "us_per_launch": k["us"],
            "copy_GBps": copy_gbps,
            "frac_of_copy": k["gbps"] / copy_gbps,
        },
        "fp32_sweep": {
            "us_back_to_back": kern["fp32"]["us"],
            "GBps_back_to_back": kern["fp32"]["gbps"],
            "us_cache_evicted": kern["fp32_cold"]["us"],
            "GBps_cache_evicted": kern["fp32_cold"]["gbps"],
            "frac_cache_evicted": kern["fp32_cold"]["gbps"] / HBM_PEAK_GBS,
            "bytes_per_launch": kern["fp32"]["bytes"],
            "note": f"the FP32 sweep's {kern['fp32']['bytes'] / 1e6:.0f} MB fit the 256 MB Infinity Cache: "
                    "back-to-back launches reuse them; the evicted figure reads 1 GiB between launches (outside "
                    "the events)",
        },
        "fp64": {
            "solves_per_s": m / fp64_t,
            "ms_per_solve": fp64_t * 1e3,
            "ms_per_solve_all": [t * 1e3 for t in res["fp64"]["times"]],
            "iterations": res["fp64"]["its"],
            "true_rel_residual": res["fp64"]["true_rel"],
            "sweep_gbps": kern["fp64"]["gbps"],
            "sweep_us": kern["fp64"]["us"],
        },
        "mixed": {
            "iterations": res["mixed"]["its"],
            "true_rel_residual": res["mixed"]["true_rel"],
            "speedup_vs_fp64": fp64_t / mixed_t,
            "ms_per_solve_all": [t * 1e3 for t in res["mixed"]["times"]],
        },
        "error_vs_reference": {
            "mixed_fwd_err": res["mixed"]["fwd_err"],
            "fp64_fwd_err": res["fp64"]["fwd_err"],
            "mixed_vs_fp64_timed_rhs": mix_vs_64,
            "reference": "exact solution x* of the manufactured problem b* = A x* (x* ~ N(0,1) seed 5, b* formed "
                         "in FP64 on the host), each path solved to 1e-8 untimed; mixed_vs_fp64 compares the two "
                         "paths' solutions of the timed right-hand side.  A relative residual of 1e-8 bounds the "
                         "forward error only by cond(A) 1e-8: both paths reach the same forward error, so the FP32 "
                         "V-cycle adds nothing to it",
        },
        "vcycle": {name: {"ms": v["ms"], "GBps": v["gbps"], "frac": v["gbps"] / HBM_PEAK_GBS} for name, v in vc.items()},
        "setup_s": setup_s,
        "autotune": tuning,
        "serving": serving,
        "oversampled": oversampled,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def oversampled_levels(agg, nb, n_cut, r, max_coarse=2048):
    """Level count and dof counts of the oversampled hierarchy: eq:sik's
    h-step s_J = min(ceil(|A_J| / n_cut), |A_J|, r) per aggregate, levels added
    until the coarsest holds at most max_coarse dofs (agg: element -> level-k
    aggregate maps of the deepest partition)."""
    sizes = np.full(agg.shape[1], nb, dtype=np.int64)
    prev = np.arange(agg.shape[1])
    dofs = [int(sizes.sum())]
    for k in range(agg.shape[0]):
        unit_of_elem = prev
        cur = agg[k]
        n_agg = int(cur.max()) + 1
        # unit -> aggregate, then |A_J| = sum of its units' sizes
        u2a = np.zeros(len(sizes), dtype=np.int64)
        u2a[unit_of_elem] = cur
        rows = np.bincount(u2a, weights=sizes, minlength=n_agg).astype(np.int64)
        sizes = np.minimum(np.minimum(np.ceil(rows / n_cut).astype(np.int64), rows), r)
        dofs.append(int(sizes.sum()))
        prev = cur
        if dofs[-1] <= max_coarse:
            return k + 2, dofs
    return agg.shape[0] + 1, dofs


def bench_oversampled(args, am, torch, dev, w, maxit):
    """The headline workload with the paper's own coarse spaces (Section 4.2):
    r = the median dofs of a level-1 aggregate, s_J per aggregate (eq:sik,
    n_cut = 3), as many levels as the coarsest level needs to hold at most
    2,048 dofs; candidates N(0,1) from seed 2.  One warm-up and args.steps
    timed solves per path, the V-cycle in both precisions, and the same with
    levels 1 and 2 matrix-free (Section 4.6, kappa = 2)."""
    agg1, _ = am.amgdg_partition_rcb(w.centroids, 2, w.params.bisections)
    r = int(np.median(np.bincount(agg1[0]) * w.A.nb))
    D = int(np.ceil(np.log2(w.mesh.n_elem)))
    deep, _ = am.amgdg_partition_rcb(w.centroids, D // w.params.bisections + 1, w.params.bisections)
    n_levels, dofs = oversampled_levels(deep, w.A.nb, w.params.n_cut, r)
    B1 = np.ascontiguousarray(np.random.default_rng(2).standard_normal((w.A.n, r)))
    out = {"r": r, "n_levels": n_levels, "levels_dofs_planned": dofs}
    b = torch.as_tensor(w.b).to(dev).contiguous()
    x = torch.zeros_like(b)
    A = w.A.to_scipy()
    for kappa in (0, 2):
        agg, _ = am.amgdg_partition_rcb(w.centroids, n_levels, w.params.bisections)
        p = am.amgdg_default_params(n_levels=n_levels, r=r, t_pre=3, t_post=3, n_cut=w.params.n_cut, mixed=1,
                                    matfree_levels=kappa)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = am.amgdg_setup(w.A.n_brow, w.A.nb, w.A.row_ptr, w.A.col_idx, w.A.vals, agg, p, B1=B1)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        infos = [am.amgdg_level_info_get(h, k) for k in range(h.n_levels)]
        res = {"setup_s": setup_s, "levels_dofs": [int(i.n_dofs) for i in infos],
               "levels_nnz": [int(i.nnzb) * i.nb * i.nb for i in infos],
               "coarse_block_sizes": [i.s for i in infos[:-1]], "hierarchy_bytes": int(infos[0].bytes_handle)}
        log(f"oversampled r={r} kappa={kappa}: setup {setup_s:.1f} s, levels {res['levels_dofs']}, "
            f"nnz {res['levels_nnz']}, {res['hierarchy_bytes'] / 1e9:.2f} GB")
        paths = (("mixed", am.AMGDG_FCG, am.AMGDG_MIXED), ("fp64", am.AMGDG_PCG, am.AMGDG_FP64))
        for name, meth, prec in (paths if kappa == 0 else paths[:1]):
            rc, st, t = _timed_solves(am, torch, h, b, x, meth, prec, maxit, max(1, min(args.steps, 2)))
            tr = float(np.linalg.norm(w.b - A @ x.cpu().numpy()) / np.linalg.norm(w.b))
            res[name] = {"iterations": st.iterations[0], "seconds": t, "solves_per_s": 1.0 / t,
                         "true_rel_residual": tr, "converged": rc == am.AMGDG_OK}
            log(f"oversampled kappa={kappa} {name}: {st.iterations[0]} iterations, {t:.2f} s, true rel {tr:.2e}")
        stream = torch.cuda.current_stream()
        res["vcycle_ms"] = {}
        for pname, prec, dt in (("fp64", am.AMGDG_FP64, torch.float64), ("fp32", am.AMGDG_MIXED, torch.float32)):
            rr = torch.randn(w.A.n, dtype=dt, device=dev)
            zz = torch.zeros_like(rr)
            for _ in range(3):
                am.amgdg_vcycle(h, rr, zz, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(10):
                am.amgdg_vcycle(h, rr, zz, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
            e1.record(stream)
            torch.cuda.synchronize()
            res["vcycle_ms"][pname] = e0.elapsed_time(e1) / 10
        log(f"oversampled kappa={kappa}: V-cycle {res['vcycle_ms']['fp64']:.3f} / {res['vcycle_ms']['fp32']:.3f} ms")
        out[f"kappa{kappa}"] = res
        h.close()
    return out


def _autotune(args, am, torch, h, m):
    """amgdg_autotune for m columns unless disabled: launch shapes that leave
    every result unchanged, plus the block-CSR lane widths with --tune-lanes;
    returns the shapes chosen per level and the seconds spent."""
    if args.no_autotune:
        return None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    am.amgdg_autotune(h, m, am.AMGDG_TUNE_LANES if args.tune_lanes else 0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    shapes = [am.amgdg_tuning_get(h, k, m) for k in range(h.n_levels - 1)]
    log(f"autotune ({dt:.2f} s): " + "; ".join(
        f"L{k} lanes {t['lanes']} cols32 {t['cols32']} mfma32 {t['mfma32']}" for k, t in enumerate(shapes)))
    return {"seconds": dt, "levels": shapes}


def _copy_bandwidth(torch, dev, stream, nbytes=2 << 30, reps=10):
    """GB/s of a plain elementwise copy of nbytes (read + write counted), far
    larger than the caches: the HBM rate a streaming kernel reaches on this part."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del src, dst
    log(f"elementwise copy of {nbytes / 1e9:.2f} GB: {2 * nbytes / t / 1e9:.0f} GB/s")
    return 2 * nbytes / t / 1e9


def _evicted_launch_time(torch, dev, stream, launch, reps, evict_bytes=1 << 30):
    """Mean duration of `launch` (one kernel) with the caches evicted before
    each launch: a 1 GiB buffer is read (summed) between launches, outside the
    event pair that brackets each launch.  A read leaves no dirty lines whose
    write-back would compete with the timed kernel."""
    buf = torch.ones(evict_bytes // 4, dtype=torch.float32, device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        buf.sum()
        e0.record(stream)
        launch()
        e1.record(stream)
    torch.cuda.synchronize()
    del buf
    return sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps * 1e-3


def _copy_calibration(args, torch, dev):
    """Three elementwise copies of a known size, for scaling HBM counters."""
    if not args.copy_calibration:
        return
    nbytes = args.copy_calibration * 1000 * 1000
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x elementwise copy of {nbytes} bytes")


def _contract(args, metric_value, ms, dtype, workload, extra):
    line = {
        "metric": "solves/sec + HBM GB/s of V-cycle to 1e-8 rel. resid; mixed vs FP64, p99 latency",
        "value": metric_value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": workload},
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


def _timed_solves(am, torch, h, b, x, method, prec, maxit, steps, restart=30, rtol=1e-8):
    """A two-iteration warm-up solve (captures the V-cycle graphs), then
    max(steps, 1) timed solves; returns the last status and the median time."""
    def one(it):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = am.amgdg_solve(h, b, x, method, prec, rtol, it, restart=restart)
        torch.cuda.synchronize()
        return rc, st, time.perf_counter() - t0
    one(2)
    times = []
    for _ in range(max(steps, 1)):
        rc, st, t = one(maxit)
        times.append(t)
    return rc, st, float(np.median(times))


def bench_convdiff(args, am, torch, dev):
    """LDG + upwind convection-diffusion, p = 2, on the Delaunay triangulation
    of 363^2 jittered points (262,088 triangles); 6-level hierarchy, r = 4,
    V(3,3); right-hand side U(-1, 1) from seed 1; right-preconditioned
    FGMRES(30) to 1e-8 with the FP64 and the FP32 V-cycle, per Peclet number."""
    from workloads import configs
    side = args.side or 363
    maxit = min(args.max_it, 5000)
    sweep = {}
    for pe in (1.0, 1e2, 1e4):
        log(f"convdiff: generating Pe = {pe:g} (side {side})")
        w = configs.convdiff2d_delaunay(side=side, peclet=pe)
        A = w.A.to_scipy()
        t0 = time.perf_counter()
        h, _ = am.setup_from_workload(w, mixed=True, restrict_resid=int(not args.no_restrict_resid))
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        infos = [am.amgdg_level_info_get(h, k) for k in range(h.n_levels)]
        log(f"convdiff Pe {pe:g}: {w.mesh.n_elem} triangles, {w.A.n} dofs, {w.A.nnzb} blocks; setup {setup_s:.2f} s; "
            f"levels n = {[i.n for i in infos]}")
        tuning = _autotune(args, am, torch, h, 1)
        b = torch.as_tensor(w.b).to(dev).contiguous()
        x = torch.zeros_like(b)
        res = {"setup_s": setup_s, "levels_n": [i.n for i in infos], "autotune": tuning}
        for name, prec in (("fp64", am.AMGDG_FP64), ("mixed", am.AMGDG_MIXED)):
            rc, st, t = _timed_solves(am, torch, h, b, x, am.AMGDG_FGMRES, prec, maxit, args.steps)
            xh = x.cpu().numpy()
            tr = float(np.linalg.norm(w.b - A @ xh) / np.linalg.norm(w.b))
            res[name] = {"iterations": st.iterations[0], "converged": rc == am.AMGDG_OK, "seconds": t,
                         "solves_per_s": 1.0 / t if rc == am.AMGDG_OK else None, "true_rel_residual": tr}
            log(f"convdiff Pe {pe:g} {name}: rc {rc}, {st.iterations[0]} iterations, {t:.2f} s, true rel {tr:.2e}")
        if pe == 1e2:
            res["kernels"] = _level0_rates(am, torch, h, infos, dev, 3)
        sweep[f"{pe:g}"] = res
        h.close()
    mid = sweep["100"]
    _contract(args, mid["fp64"]["solves_per_s"], mid["fp64"]["seconds"] * 1e3, "f64 (and f32 V-cycle + f64 Krylov)",
              f"2D convection-diffusion, LDG + upwind p=2 on the Delaunay triangulation of {side}^2 jittered points, "
              f"6-level RCB hierarchy, r=4, V(3,3), FGMRES(30) to 1e-8; value: FP64 at Peclet 100",
              {"peclet_sweep": sweep, "max_it": maxit})


# Iteration counts printed in Section 5.1 for this problem (solver / pCG, IP / LDG).
PAPER_HEX_ITERATIONS = {3: {"ip": 7, "ldg": 7, "ip_pcg": 6, "ldg_pcg": 6},
                        4: {"ip": 7, "ldg": 8, "ip_pcg": 6, "ldg_pcg": 7},
                        5: {"ip": 7, "ldg": 9, "ip_pcg": 6, "ldg_pcg": 7}}
# Section 5.2 (LDG, M = 4): iterations as the solver and as the CG preconditioner,
# h*-multigrid (an intra-element step first) and h-multigrid, per degree p
PAPER_HEX_HP = {1: {"hstar": 8, "h": 8, "hstar_pcg": 7, "h_pcg": 6},
                2: {"hstar": 8, "h": 9, "hstar_pcg": 6, "h_pcg": 7},
                3: {"hstar": 10, "h": 9, "hstar_pcg": 7, "h_pcg": 7}}


def bench_hex(args, am, torch, dev):
    """The structured Poisson problem of Section 5.1: 2^M cubes per direction of
    [-1, 1]^3, Q_p, IP (penalty M (p+1)^2 / 2) and minimal-dissipation LDG,
    Dirichlet on x = -1 and Neumann elsewhere, right-hand side of the paper's
    manufactured solution; ceil(log_8 |T_h|) levels of 8-way RCB aggregates
    (one more with an h*-step first), r candidates (coarse sizes
    min(ceil(|A_J| / 6), |A_J|, r) per aggregate), V(3,3); multigrid as the
    solver and as the CG preconditioner, to the paper's 1e-7, in FP64, and
    flexible CG with the FP32 V-cycle.  Every (r, M, flux, p, h*, kappa)
    combination asked for is one row of the table: iterations beside the
    paper's, times, the hierarchy (dofs, nonzeros, device bytes), the V-cycle's
    time in both precisions; kappa > 0 applies levels 1..kappa matrix-free."""
    from workloads import configs
    maxit = min(args.max_it, 2000)
    table = {}
    for r in args.hex_r:
        for M in args.hex_m:
            for flux in args.hex_flux:
                for p in args.hex_p:
                    for hstar in ([False, True] if args.hex_hstar and p >= 2 else [False]):
                        for kappa in args.hex_matfree:
                            w = configs.poisson3d_hex(M, p=p, flux=flux, r=r, hstar=hstar)
                            if kappa > w.params.n_levels - 2:
                                continue
                            key = f"M{M}_{flux}_r{r}" + (f"_p{p}" if p != 1 else "") + ("_hstar" if hstar else "") \
                                + (f"_mf{kappa}" if kappa else "")
                            table[key] = _hex_row(args, am, torch, dev, w, M, flux, r, p, hstar, kappa, maxit)
    extra = {"hex_table": table, "max_it": maxit}
    if not args.no_cpu_baseline:
        extra["cpu_baseline"] = _hex_cpu_baseline(configs, table)
    key = "M5_ip_r16" if "M5_ip_r16" in table else next(iter(table))
    top = table[key]["pcg"]
    _contract(args, 1.0 / top["seconds"], top["seconds"] * 1e3, "f64 (and f32 V-cycle + f64 Krylov)",
              "3D Poisson on 2^M hexahedra per direction of [-1,1]^3, Q_p, IP and LDG, Dirichlet x=-1, "
              "Neumann elsewhere, paper's manufactured solution, ceil(log_8 |T_h|) levels, V(3,3), "
              f"to 1e-7; value: FP64 multigrid-preconditioned CG, {key}", extra)


def _hex_row(args, am, torch, dev, w, M, flux, r, p, hstar, kappa, maxit):
    A = w.A.to_scipy()
    t0 = time.perf_counter()
    h, _ = am.setup_from_workload(w, mixed=True, matfree_levels=kappa,
                                  restrict_resid=int(not args.no_restrict_resid))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    infos = [am.amgdg_level_info_get(h, k) for k in range(h.n_levels)]
    b = torch.as_tensor(w.b).to(dev).contiguous()
    x = torch.zeros_like(b)
    tag = f"hex M={M} {flux} p={p} r={r}{' h*' if hstar else ''}{f' kappa={kappa}' if kappa else ''}"
    res = {"dofs": w.A.n, "p": p, "hstar": hstar, "matfree_levels": kappa, "setup_s": setup_s,
           "levels_dofs": [int(i.n_dofs) for i in infos],
           "levels_nnz": [int(i.nnzb) * i.nb * i.nb for i in infos],
           "levels_stored": [not i.matfree for i in infos],
           "coarse_block_sizes": [i.s for i in infos[:-1]],
           "hierarchy_bytes": int(infos[0].bytes_handle)}
    for name, meth, prec in (("solver", am.AMGDG_STATIONARY, am.AMGDG_FP64),
                             ("pcg", am.AMGDG_PCG, am.AMGDG_FP64),
                             ("fcg_mixed", am.AMGDG_FCG, am.AMGDG_MIXED)):
        rc, st, t = _timed_solves(am, torch, h, b, x, meth, prec, maxit, args.steps, rtol=1e-7)
        tr = float(np.linalg.norm(w.b - A @ x.cpu().numpy()) / np.linalg.norm(w.b))
        res[name] = {"iterations": st.iterations[0], "converged": rc == am.AMGDG_OK, "seconds": t,
                     "true_rel_residual": tr}
        log(f"{tag} {name}: rc {rc}, {st.iterations[0]} iterations, {t * 1e3:.1f} ms, true rel {tr:.2e}")
    res["vcycle_ms"] = {}
    stream = torch.cuda.current_stream()
    for pname, prec, dt in (("fp64", am.AMGDG_FP64, torch.float64), ("fp32", am.AMGDG_MIXED, torch.float32)):
        rr = torch.randn(w.A.n, dtype=dt, device=dev)
        zz = torch.zeros_like(rr)
        for _ in range(3):
            am.amgdg_vcycle(h, rr, zz, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            am.amgdg_vcycle(h, rr, zz, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e1.record(stream)
        torch.cuda.synchronize()
        res["vcycle_ms"][pname] = e0.elapsed_time(e1) / 20
    log(f"{tag}: levels {res['levels_dofs']}, nnz {res['levels_nnz']}, {res['hierarchy_bytes'] / 1e6:.1f} MB, "
        f"V-cycle {res['vcycle_ms']['fp64']:.3f} / {res['vcycle_ms']['fp32']:.3f} ms (FP64 / FP32)")
    if p == 1 and not hstar and M in PAPER_HEX_ITERATIONS:
        paper = PAPER_HEX_ITERATIONS[M]
        res["paper_iterations"] = {"solver": paper[flux], "pcg": paper[flux + "_pcg"]}
    elif M == 4 and flux == "ldg" and p in PAPER_HEX_HP:
        pp = PAPER_HEX_HP[p]
        k = "hstar" if hstar else "h"
        res["paper_iterations"] = {"solver": pp[k], "pcg": pp[k + "_pcg"]}
    if M == 5 and r == 16 and p == 1 and not kappa:
        res["kernels"] = _level0_rates(am, torch, h, infos, dev, 3)
    h.close()
    return res


def _hex_cpu_baseline(configs, table, M=4, flux="ldg", r=16):
    """The FP64 oracle on the host cores, one whole pCG solve to 1e-7 of the hex
    problem at M = 4 (LDG, r = 16), beside the GPU's time for the same solve."""
    from threadpoolctl import threadpool_info

    from oracle import amg, krylov, rcb
    w = configs.poisson3d_hex(M, flux=flux, r=r)
    log(f"cpu baseline (hex M={M} {flux} r={r}): oracle setup")
    t0 = time.perf_counter()
    aggs, _ = rcb.rcb_hierarchy(w.centroids, w.params.n_levels, w.params.bisections)
    A = w.A.to_scipy()
    H = amg.setup(A, w.A.nb, aggs, w.params, w.B1)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, its, _ = krylov.pcg(A, w.b, lambda v: amg.vcycle(H, v), 1e-7, 500)[:3]
    t_solve = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    gpu = table.get(f"M{M}_{flux}_r{r}", {}).get("pcg")
    log(f"cpu baseline (hex): setup {t_setup:.1f} s, pCG {its} iterations in {t_solve:.2f} s")
    return {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"FP64 oracle (NumPy/SciPy): one whole pCG solve to 1e-7 of the hex problem at M={M}, {flux}, "
                  f"r={r} ({its} iterations, {t_solve:.2f} s; setup {t_setup:.1f} s not counted); sparse products "
                  f"single-threaded, dense LAPACK on {threads} threads",
        "gpu_seconds_same_solve": gpu["seconds"] if gpu else None,
        "gpu_iterations_same_solve": gpu["iterations"] if gpu else None,
    }


def _level0_rates(am, torch, h, infos, dev, nu, m=1, reps=20):
    """HIP-event times of the V-cycle and of the level-0 sweep on D^-1 A (FP32
    and FP64, m columns, internal order) with their algorithmic GB/s."""
    stream = torch.cuda.current_stream()
    out = {}
    n = infos[0].n
    for name, (prec, wb, dt) in {"fp32": (am.AMGDG_MIXED, 4, torch.float32),
                                 "fp64": (am.AMGDG_FP64, 8, torch.float64)}.items():
        shape = (n,) if m == 1 else (n, m)
        r = torch.randn(shape, dtype=dt, device=dev)
        z = torch.zeros_like(r)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            am.amgdg_vcycle(h, r, z, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e0.record(stream)
        for _ in range(reps):
            am.amgdg_vcycle(h, r, z, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e1.record(stream)
        torch.cuda.synchronize()
        tv = e0.elapsed_time(e1) / reps * 1e-3
        nN = infos[-1].n
        bv = sum(level_bytes(i, wb, m, nu) for i in infos[:-1]) + nN * nN * 8 + 2 * nN * m * 8
        xx, bb, yy = torch.randn_like(r), torch.randn_like(r), torch.zeros_like(r)
        for _ in range(3):
            am.amgdg_apply(h, 0, am.AMGDG_OP_SWEEP_SCALED, xx, bb, yy, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e0.record(stream)
        for _ in range(reps):
            am.amgdg_apply(h, 0, am.AMGDG_OP_SWEEP_SCALED, xx, bb, yy, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e1.record(stream)
        torch.cuda.synchronize()
        ts = e0.elapsed_time(e1) / reps * 1e-3
        sb = sweep_bytes(infos[0], wb, m)
        out[name] = {"vcycle_ms": tv * 1e3, "vcycle_GBps": bv / tv / 1e9, "sweep_us": ts * 1e6,
                     "sweep_GBps": sb / ts / 1e9, "sweep_frac": sb / ts / 1e9 / HBM_PEAK_GBS, "sweep_bytes": sb}
        log(f"level-0 sweep {name}: {ts * 1e6:.1f} us ({sb / ts / 1e9:.0f} GB/s, {sb / 1e6:.1f} MB); "
            f"V-cycle {tv * 1e3:.3f} ms ({bv / tv / 1e9:.0f} GB/s)")
        del r, z, xx, bb, yy
    return out


def bench_poisson3d(args, am, torch, dev):
    """3D Poisson, SIPG p = 2 on 64^3 cube cells x 6 Kuhn tetrahedra with vertex
    jitter 0.2h (1,572,864 tets, 15,728,640 dofs); 5-level hierarchy, r = 4,
    V(2,2); 16 right-hand sides N(0,1) from seed 1 solved together (every
    kernel of the V-cycle and the Krylov loop handles the 16 columns in one
    launch) to 1e-8: FP32 V-cycle in FP64 flexible CG, and FP64 CG."""
    from workloads import configs
    cells = args.side or 64
    m = 16
    maxit = args.max_it
    log(f"poisson3d: generating {cells}^3 x 6 tetrahedra, {m} right-hand sides")
    t0 = time.perf_counter()
    w = configs.poisson3d_kuhn(n=cells, n_rhs=m, log=log)
    log(f"poisson3d: {w.mesh.n_elem} tets, {w.A.n} dofs, {w.A.nnzb} blocks ({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    h, _ = am.setup_from_workload(w, mixed=True, restrict_resid=int(not args.no_restrict_resid))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    infos = [am.amgdg_level_info_get(h, k) for k in range(h.n_levels)]
    log(f"poisson3d: setup {setup_s:.2f} s; levels n = {[i.n for i in infos]}, "
        f"omega = {[round(i.omega, 4) for i in infos[:-1]]}")
    tuning = _autotune(args, am, torch, h, m)
    b = torch.as_tensor(w.b).to(dev).contiguous()
    w.b = None
    x = torch.zeros_like(b)
    y = torch.zeros_like(b)
    res = {}
    paths = [("mixed", am.AMGDG_FCG, am.AMGDG_MIXED)]
    if not args.skip_fp64:
        paths.append(("fp64", am.AMGDG_PCG, am.AMGDG_FP64))
    for name, meth, prec in paths:
        rc, st, t = _timed_solves(am, torch, h, b, x, meth, prec, maxit, args.steps)
        am.amgdg_apply(h, 0, am.AMGDG_OP_RESIDUAL, x, b, y)
        tr = float((torch.linalg.norm(y, dim=0) / torch.linalg.norm(b, dim=0)).max())
        res[name] = {"iterations_max": st.max_iterations, "converged": rc == am.AMGDG_OK, "seconds": t,
                     "solves_per_s": m / t if rc == am.AMGDG_OK else None, "true_rel_residual_max": tr}
        log(f"poisson3d {name}: rc {rc}, {st.max_iterations} iterations, {t:.2f} s, max true rel {tr:.2e}")
    nu = 2
    stream = torch.cuda.current_stream()
    vc = {}
    for name, (prec, wb, dt) in {"fp32": (am.AMGDG_MIXED, 4, torch.float32),
                                 "fp64": (am.AMGDG_FP64, 8, torch.float64)}.items():
        r = torch.randn(b.shape, dtype=dt, device=dev)
        z = torch.zeros_like(r)
        for _ in range(2):
            am.amgdg_vcycle(h, r, z, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reps = 5
        for _ in range(reps):
            am.amgdg_vcycle(h, r, z, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps * 1e-3
        nN = infos[-1].n
        byts = sum(level_bytes(i, wb, m, nu) for i in infos[:-1]) + nN * nN * 8 + 2 * nN * m * 8
        xx, bb, yy = torch.randn_like(r), torch.randn_like(r), torch.zeros_like(r)
        for _ in range(2):
            am.amgdg_apply(h, 0, am.AMGDG_OP_SWEEP_SCALED, xx, bb, yy, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e0.record(stream)
        for _ in range(reps):
            am.amgdg_apply(h, 0, am.AMGDG_OP_SWEEP_SCALED, xx, bb, yy, precision=prec, flags=am.AMGDG_INTERNAL_ORDER)
        e1.record(stream)
        torch.cuda.synchronize()
        ts = e0.elapsed_time(e1) / reps * 1e-3
        sb = sweep_bytes(infos[0], wb, m)
        vc[name] = {"vcycle_ms": t * 1e3, "vcycle_GBps": byts / t / 1e9, "sweep_us": ts * 1e6,
                    "sweep_GBps": sb / ts / 1e9, "sweep_frac": sb / ts / 1e9 / HBM_PEAK_GBS}
        log(f"poisson3d V-cycle {name}: {t * 1e3:.2f} ms ({byts / t / 1e9:.0f} GB/s); level-0 sweep "
            f"{ts * 1e6:.0f} us ({sb / ts / 1e9:.0f} GB/s)")
        del r, z, xx, bb, yy
    _copy_calibration(args, torch, dev)
    mx = res["mixed"]
    _contract(args, mx["solves_per_s"], mx["seconds"] * 1e3, "f32 V-cycle + f64 Krylov",
              f"3D Poisson SIPG p=2 on {cells}^3 x 6 jittered Kuhn tetrahedra ({infos[0].n_units} tets, "
              f"{infos[0].n} dofs), 5-level RCB hierarchy, r=4, V(2,2), {m} RHS per solve, tol 1e-8",
              {"solves": res, "kernels_m16": vc, "setup_s": setup_s, "levels_n": [i.n for i in infos],
               "autotune": tuning})


def bench_serving_stream(args, am, torch, dev):
    """Serving stream: a catalogue of operator instances (2D jittered Delaunay
    meshes, 1k-200k triangles, p = 1..4, SIPG-Poisson or LDG-upwind
    convection-diffusion) with hierarchies resident on the device; solve
    requests arrive as a Poisson process (exponential gaps, seed 4), each a
    uniform pick from the catalogue with a fresh right-hand side (seed 10000 +
    request).  SIPG requests run flexible CG, LDG requests FGMRES(30), both
    with the FP32 V-cycle, to 1e-8.  Requests arriving in the warm-up window
    are served but not counted."""
    from workloads import configs
    log(f"serving: generating {args.catalogue} operators (up to {args.t_max:g} triangles)")
    cat = configs.serving_catalogue(n_ops=args.catalogue, t_max=args.t_max, log=log)
    handles, setup_s = [], []
    for w in cat:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, _ = am.setup_from_workload(w, mixed=True, restrict_resid=int(not args.no_restrict_resid))
        torch.cuda.synchronize()
        setup_s.append(time.perf_counter() - t0)
        handles.append(h)
    log(f"serving: {len(cat)} hierarchies set up, {sum(setup_s):.1f} s in total")
    rate = args.serve_rate if args.serve_rate > 0 else 20.0
    horizon = args.serve_warmup + args.serve_duration
    rng = np.random.default_rng(4)
    t_arr, picks = [], []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > horizon:
            break
        t_arr.append(t)
        picks.append(int(rng.integers(0, len(cat))))
    n_req = len(t_arr)
    srv = am.Server(width=args.serve_width, hbm_budget_bytes=int(args.budget_gb * (1 << 30)))
    maxit = min(args.max_it, 20000)
    out = {}
    keep = {}
    stream = torch.cuda.current_stream()
    nxt = 0
    log(f"serving: {n_req} requests at {rate:g}/s over {horizon:g} s")
    t0 = time.perf_counter()
    last_log = t0
    while len(out) < n_req:
        now = time.perf_counter() - t0
        while nxt < n_req and t_arr[nxt] <= now:
            w = cat[picks[nxt]]
            g = np.random.default_rng(10000 + nxt)
            bh = g.standard_normal(w.A.n) if w.krylov == "pcg" else g.uniform(-1.0, 1.0, w.A.n)
            b = torch.as_tensor(bh).to(dev)
            x = torch.zeros_like(b)
            stream.synchronize()
            meth = am.AMGDG_FCG if w.krylov == "pcg" else am.AMGDG_FGMRES
            srv.submit(handles[picks[nxt]], b, x, meth, am.AMGDG_MIXED, 1e-8, maxit, restart=30, tag=nxt)
            keep[nxt] = (b, x)
            nxt += 1
        srv.step(wait=nxt == n_req)
        for tag, status, its, relres, lat in srv.poll(256):
            out[tag] = (status, its, relres, lat)
            keep.pop(tag, None)
        if time.perf_counter() - last_log > 10.0:
            last_log = time.perf_counter()
            log(f"serving: t = {last_log - t0:.0f} s, {nxt} submitted, {len(out)} done")
    makespan = time.perf_counter() - t0
    srv.close()
    counted = [i for i in range(n_req) if t_arr[i] >= args.serve_warmup]
    lat = np.array([out[i][3] for i in counted])
    done_in = [i for i in counted if t_arr[i] + out[i][3] <= horizon]
    conv = sum(1 for i in counted if out[i][0] == am.AMGDG_OK)
    by_kind = {}
    for kind in ("pcg", "gmres"):
        ids = [i for i in counted if cat[picks[i]].krylov == kind]
        if ids:
            by_kind["sipg_fcg" if kind == "pcg" else "ldg_fgmres"] = {
                "requests": len(ids), "mean_iterations": float(np.mean([out[i][1] for i in ids])),
                "p50_latency_s": float(np.percentile([out[i][3] for i in ids], 50)),
                "p99_latency_s": float(np.percentile([out[i][3] for i in ids], 99))}
    res = {
        "catalogue": [{"name": w.name, "dofs": w.A.n, "levels": w.params.n_levels, "setup_s": st}
                      for w, st in zip(cat, setup_s)],
        "arrival_rate_per_s": rate, "warmup_s": args.serve_warmup, "duration_s": args.serve_duration,
        "requests_counted": len(counted), "converged": conv,
        "completed_per_s": len(done_in) / args.serve_duration,
        "throughput_solves_per_s": n_req / makespan, "makespan_s": makespan,
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "by_kind": by_kind, "batch_width": args.serve_width, "budget_gb": args.budget_gb,
    }
    for hnd in handles:
        hnd.close()
    log(f"serving: {len(counted)} counted requests, {conv} converged, p50 {res['p50_latency_s']:.3f} s, "
        f"p99 {res['p99_latency_s']:.3f} s, {n_req / makespan:.1f} solves/s over {makespan:.1f} s")
    _contract(args, res["throughput_solves_per_s"], 1e3 / max(res["throughput_solves_per_s"], 1e-12),
              "f32 V-cycle + f64 Krylov",
              f"serving stream: {len(cat)} operators (2D jittered Delaunay, up to {args.t_max:g} triangles, p=1..4, "
              f"SIPG flexible CG / LDG-upwind FGMRES(30)), Poisson arrivals at {rate:g}/s, tol 1e-8",
              {"serving": res})


def serve_bench(am, h, n, dev, n_req, width, rate, maxit):
    """Continuous batching: n_req single-RHS requests (mixed FCG to 1e-8,
    right-hand sides standard normal, seeds 1000 + i) through one server of
    batches of `width` columns; all at once (rate 0) or with Poisson arrivals.
    Latency runs from submission to the step that saw x written."""
    import numpy as np
    import torch
    B = [torch.as_tensor(np.random.default_rng(1000 + i).standard_normal(n)).to(dev).contiguous()
         for i in range(n_req)]
    X = [torch.zeros_like(b) for b in B]
    gaps = np.random.default_rng(7).exponential(1.0 / rate, n_req) if rate > 0 else np.zeros(n_req)
    arrive = np.cumsum(gaps) - gaps[0]
    torch.cuda.synchronize()
    srv = am.Server(width=width, hbm_budget_bytes=64 << 30)
    log(f"serving: {n_req} requests, batch width {width}, "
        f"{'all at once' if rate <= 0 else f'Poisson arrivals at {rate} /s'}")
    out = {}
    nxt = 0
    t0 = time.perf_counter()
    while len(out) < n_req:
        now = time.perf_counter() - t0
        while nxt < n_req and arrive[nxt] <= now:
            srv.submit(h, B[nxt], X[nxt], am.AMGDG_FCG, am.AMGDG_MIXED, 1e-8, maxit, tag=nxt)
            nxt += 1
        srv.step(wait=nxt == n_req)
        for tag, status, its, rel, lat in srv.poll():
            out[tag] = (status, its, rel, lat)
            log(f"serving: request {tag} done, status {status}, {its} iterations, {lat:.2f} s")
    makespan = time.perf_counter() - t0
    srv.close()
    lat = np.array([out[i][3] for i in range(n_req)])
    its = np.array([out[i][1] for i in range(n_req)])
    return {
        "requests": n_req,
        "batch_width": width,
        "arrivals": "all at t=0" if rate <= 0 else f"Poisson, {rate} requests/s",
        "solves_per_s": n_req / makespan,
        "makespan_s": makespan,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_iterations": float(its.mean()),
        "all_converged": bool(all(out[i][0] == am.AMGDG_OK and out[i][2] <= 1e-8 for i in range(n_req))),
        "batch_bytes": am.amgdg_batch_bytes(h, width),
    }


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, gpu_iterations, n_iter=5):
    """The FP64 oracle on the host cores: its setup, then n_iter PCG iterations
    at full size, extrapolated to the GPU's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import amg, krylov, rcb
    log("cpu baseline: oracle setup")
    t0 = time.perf_counter()
    aggs, _ = rcb.rcb_hierarchy(w.centroids, w.params.n_levels, w.params.bisections)
    A = w.A.to_scipy()
    H = amg.setup(A, w.A.nb, aggs, w.params, w.B1)
    t_setup = time.perf_counter() - t0
    b = w.b if w.b.ndim == 1 else w.b[:, 0]
    log(f"cpu baseline: oracle setup {t_setup:.1f} s; timing {n_iter} PCG iterations")
    t0 = time.perf_counter()
    krylov.pcg(A, b, lambda r: amg.vcycle(H, r), 1e-30, n_iter)
    t_it = (time.perf_counter() - t0) / n_iter
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {
        "value": 1.0 / (t_it * gpu_iterations),
        "unit": "solves/s",
        "cores": threads,
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": f"FP64 oracle (NumPy/SciPy) setup ({t_setup:.1f} s) then {n_iter} PCG iterations on the full "
                  f"workload ({t_it:.3f} s each), extrapolated to the {gpu_iterations} iterations of one solve; "
                  f"sparse products single-threaded, dense LAPACK on {threads} threads",
    }


if __name__ == "__main__":
    main()
