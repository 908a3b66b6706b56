"""Benchmark: time-to-solution and DOF/s of the clamped variable-coefficient 3-D biharmonic
solve on one MI355X (mixed precision: FP32 transforms inside FP64 refinement), next to the
plain FP64 GPU form, with the DST pass kernel's roofline and the CPU oracle as baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 1024] [--no-fp64] [--no-cpu]

A step is one whole solve (ConstructSchurRHS, preconditioned GMRES with Schur matvecs,
recovery, and for the mixed form the FP64 refinement sweeps) of the synthetic problem with
inputs resident in HBM; both forms solve to the same Schur residual tolerance, and their
errors are measured against an untimed FP64 solve at 1e-13.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solve time + DOF/s at 1024^3 to 1e-10 rel err, mixed vs FP64; DST HBM GB/s"


def _pmc_traffic(kernel_src_hash):
    """Measured HBM bytes per DST pass launch from the committed rocprofv3 PMC summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "dst_pass_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("dst_source_sha1") != kernel_src_hash:
        return None
    try:
        return {"fetch_bytes": float(kv["fetch_bytes_per_launch"]), "write_bytes": float(kv["write_bytes_per_launch"]),
                "n": int(kv["n"])}
    except (KeyError, ValueError):
        return None


def _src_hash():
    """Hash of the sources of the DST pass kernels (the PMC summary is valid for these)."""
    h = hashlib.sha1()
    for f in ("dst_fast.hip", "dst_pipe.hip", "dst_device.h"):
        h.update(open(os.path.join(ROOT, "paper_2609_16478_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def cpu_baseline(n=128, tol=1e-10, dim=3):
    """The oracle's Algorithm-1 tier (scipy DST-I, numpy stencils, FP64 GMRES(30), no
    preconditioner) on the benchmark's 3-D problem at n^3 (dim = 2: the 2-D variable-
    coefficient problem at n^2) -- a configuration the line also reports GPU times for
    (gpu_same_config) -- timed on this host's cores."""
    import numpy as np
    import workloads as W
    from oracle import fast
    cores = len(os.sched_getaffinity(0))
    p = W.config3(n) if dim == 3 else W.config2(n)
    t0 = time.perf_counter()
    ft = fast.FastTier(p, workers=cores)
    U, V, Q, info = ft.solve(tol=tol)
    dt = time.perf_counter() - t0
    err = float(np.abs(U - p.u_exact).max() / np.abs(p.u_exact).max())
    what = "the benchmark's 3-D problem" if dim == 3 else "the 2-D variable-coefficient problem"
    return {"value": n ** dim / dt, "unit": "DOF/s", "cores": cores, "kind": "oracle",
            "sample": f"one whole FP64 fast-tier solve (scipy DST-I with workers={cores}, numpy stencils, "
                      f"own GMRES(30) without preconditioner, Schur tol {tol:g}) of {what} "
                      f"at n={n} ({info['iters']} GMRES iterations, {dt:.1f} s, rel err vs exact {err:.2e}); "
                      f"DOF = n^{dim}; the GPU's times for this configuration are in config.gpu_same_config"
                      + ("" if dim == 3 else "_2d"),
            "time_s": dt, "n": n}


def gpu_same_config(ah, W, torch, dev, n, tol, steps=3, dim=3):
    """GPU solve times of a CPU baseline's configuration (the 3-D problem at n^3, or with
    dim = 2 the 2-D one at n^2, the same Schur tolerance), both forms, after a warm-up solve;
    setup excluded."""
    prob = W.config3(n, xp="torch", device=dev) if dim == 3 else W.config2(n, xp="torch", device=dev)
    out = {"n": n, "dim": dim, "tol": tol}
    for name, prec in (("mixed", ah.MIXED), ("fp64", ah.FP64)):
        with ah.Solver(prob, precision=prec, tol=tol) as s:
            s.solve()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                _, _, _, st = s.solve()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / steps
        out[name] = {"ms": dt * 1e3, "dof_per_s": n ** dim / dt, "gmres_iters": st.gmres_iters}
    return out


def _pitch(n):
    return (n - 1 + 31) // 32 * 32


def _pattern_copies(ah, torch, dev, n, reps=5):
    """GB/s (read + write) of the library's calibration copies over an FP32 volume of the
    solver's interior work-array shape [n-1][n-1][pitch]: linear, y-pass tiles, z-pass tiles."""
    x = torch.zeros(n - 1, n - 1, _pitch(n), dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    out = {}
    for name, pattern in (("linear", 0), ("y_tiles", 1), ("z_tiles", 2)):
        ah.copy_bandwidth(pattern, x, y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ah.copy_bandwidth(pattern, x, y)
        e1.record()
        torch.cuda.synchronize()
        out[name] = reps * 2 * x.numel() * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del x, y
    return out


def _varbeta(ah, W, torch, dev, n):
    """One FP64 solve of Example 2 with its variable alpha and beta (BiCGSTAB V-solves), a
    warm-up solve first; the kernel-class times come from HIP events on the solve stream."""
    prob = W.example2(n, 5.0, 1.0, xp="torch", device=dev, chunk=32)
    prob.v_exact = None
    with ah.Solver(prob, precision=ah.FP64, tol=1e-12) as s:
        s.solve()
        s.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, _, _, st = s.solve()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = s.kernel_times()
    err = (u - prob.u_exact).abs().max().item()
    print(f"[bench] variable beta n={n}: {1e3 * (t1 - t0):.1f} ms, {st.gmres_iters} GMRES, {st.vsolve_iters} "
          f"BiCGSTAB, err {err:.3e}", file=sys.stderr, flush=True)
    return {"metric": "FP64 solve time, Example 2 with variable alpha and beta", "n": n, "ms": 1e3 * (t1 - t0),
            "gmres_iters": st.gmres_iters, "bicgstab_iters": st.vsolve_iters, "err_u_inf": err,
            "kernel_classes_ms": {k: v[0] for k, v in kt.items() if v[1]},
            "kernel_classes_launches": {k: v[1] for k, v in kt.items() if v[1]}}


def _paper_timing(ah, W, torch, dev):
    """The workloads of the paper's timing table: the classical biharmonic equation (alpha = 1,
    beta = 0) with the solutions of Example 2 ((q, p) = (5, 1)) and of the oscillatory example
    (k = (25, 5, 25)), clamped at x = 0 and Navier elsewhere (the setting of the paper's
    convergence tests; the table does not restate it).  Setup (coefficients, tables, kernel
    choice) and solve are timed separately with the device synchronised, FP64 and mixed, each
    to a Schur tolerance of h^3.5; the error is against the exact solution.  Handle memory
    comes from PyTorch's caching allocator, whose cache is kept between the solvers as in a
    process that solves repeatedly: device memory handed back to the device runtime and requested
    again moments later can take up to seconds per multi-GiB block to map.  (16-thread CPU
    times in the paper: context only.)"""
    out = {"metric": "setup + solve seconds of the paper's timing-table workloads, Schur tol h^3.5",
           "unit": "s", "cases": []}
    makers = {"example2_q5_p1": lambda n: W.example2(n, 5.0, 1.0, alpha="1", beta=0.0, xp="torch", device=dev,
                                                     chunk=32),
              "example3_k25_5_25": lambda n: W.example3(n, (25.0, 5.0, 25.0), alpha="1", beta=0.0, xp="torch",
                                                        device=dev, chunk=32)}
    for name, mk in makers.items():
        for n in (128, 256, 512, 1024):
            prob = mk(n)
            prob.v_exact = None
            for prec, pname in ((ah.FP64, "fp64"), (ah.MIXED, "mixed")):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s = ah.Solver(prob, precision=prec, tol=(1.0 / n) ** 3.5)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                u, _, _, st = s.solve()
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                s.close()
                err = (u - prob.u_exact).abs().max().item()
                rec = {"example": name, "n": n, "precision": pname, "setup_s": t1 - t0, "solve_s": t2 - t1,
                       "gmres_iters": st.gmres_iters, "sweeps": st.sweeps, "converged": st.converged,
                       "err_u_inf": err}
                out["cases"].append(rec)
                print(f"[bench] {name} n={n} {pname}: setup {t1 - t0:.3f} s, solve {t2 - t1:.3f} s, "
                      f"{st.gmres_iters} GMRES, err {err:.3e}", file=sys.stderr, flush=True)
                del u, s
            del prob
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-n2d", type=int, default=1024,
                    help="grid of the second CPU-vs-GPU configuration (2-D variable-coefficient problem)")
    ap.add_argument("--cpu-n", type=int, default=128,
                    help="grid of the CPU oracle baseline (and of the GPU times reported beside it)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-10,
                    help="relative Schur residual both forms solve to (FP64 GMRES tolerance and the "
                         "mixed form's refinement stop)")
    ap.add_argument("--profile-matvec", type=int, default=0,
                    help="profiling target: set up the mixed-precision handle and run this many "
                         "Schur matvecs, then exit (no JSON line)")
    ap.add_argument("--profile-prec", choices=("mixed", "fp64"), default="mixed",
                    help="operator precision of --profile-matvec (mixed = the FP32 operator)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="profiling target: three plain 2 GiB device copies (counter calibration)")
    ap.add_argument("--dst-compare", action="store_true",
                    help="profiling target: contiguous and strided DST-I passes over 2^20 pencils of "
                         "N-1 = 31, 63, 127 points in FP32 and FP64, three each with the FFT kernels "
                         "and three with the matrix-core products")
    ap.add_argument("--profile-solve", action="store_true",
                    help="profiling target: one warm-up and one timed solve of the benchmark problem in "
                         "the --profile-prec form (tolerance --tol), 0.3 s apart so that a kernel trace "
                         "separates them, then exit (no JSON line)")
    ap.add_argument("--no-instance-loop", action="store_true",
                    help="skip the per-instance FP64 loop over the batched workload")
    ap.add_argument("--batch-profile", type=int, default=0,
                    help="profiling target: set up the 512-instance 2-D batch and run this many mixed "
                         "batched solves after a warm-up, then exit (no JSON line)")
    ap.add_argument("--varbeta", type=int, default=0,
                    help="separate target: one FP64 solve of Example 2 with its variable alpha and beta "
                         "((q, p) = (5, 1), the workload of Table 2) at this n^3, tolerance 1e-12, with the "
                         "kernel-class times; prints one JSON line")
    ap.add_argument("--paper-timing", action="store_true",
                    help="separate target: the workloads of the paper's timing table (the classical "
                         "biharmonic equation, alpha = 1, beta = 0, with the solutions of Example 2, (q, p) "
                         "= (5, 1), and of the oscillatory example, k = (25, 5, 25); clamped at x = 0, Navier "
                         "elsewhere) at 128^3 ... 1024^3, FP64 and mixed, to a Schur tolerance of h^3.5; "
                         "prints one JSON line with setup and solve times")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver has no "
              "multi-GPU path (batches would split by instance, a single volume into z slabs with an "
              "all-to-all around each z pass).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_16478_amd as ah
    import workloads as W

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        x = torch.ones(2 ** 28, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 copies of {x.numel() * 8} bytes", file=sys.stderr)
        gb = _pattern_copies(ah, torch, dev, args.n)
        print(f"[bench] calibration copies of the {args.n - 1}^2 x {_pitch(args.n)} FP32 volume: "
              + ", ".join(f"{k} {v:.0f} GB/s" for k, v in gb.items()), file=sys.stderr)
        return
    if args.dst_compare:
        for N in (32, 64, 128):
            for dt, p in ((torch.float32, ah.MIXED), (torch.float64, ah.FP64)):
                g = torch.Generator(device=dev).manual_seed(N)
                xr = torch.randn(1024, 1024, N - 1, dtype=dt, device=dev, generator=g)
                xs = torch.randn(1024, N - 1, 1024, dtype=dt, device=dev, generator=g)
                for var in (5, 4):  # FFT kernels only, then the matrix-core products
                    ah.set_dst_variant(var)
                    for _ in range(3):
                        ah.dst1(xr, 0, p)
                        ah.dst1(xs, 1, p)
                    torch.cuda.synchronize()
                ah.set_dst_variant(0)
                del xr, xs
                print(f"[bench] dst compare N={N} {dt}: 2^20 pencils, contiguous and strided", file=sys.stderr,
                      flush=True)
        return
    if args.paper_timing:
        print(json.dumps(_paper_timing(ah, W, torch, dev)))
        return
    if args.varbeta:
        print(json.dumps(_varbeta(ah, W, torch, dev, args.varbeta)))
        return
    if args.batch_profile:
        specs = W.config4_specs(args.batch_count)
        bprobs = [W.config4_instance(sp, xp="torch", device=dev, with_exact=False) for sp in specs]
        ah.solve_batched(bprobs, precision=ah.MIXED, tol=args.tol)
        # a calibration copy (kernel k_copy_linear) before each timed batch and after the last
        # marks the batch windows in a kernel trace
        mark = torch.zeros(1, 1, 32, dtype=torch.float32, device=dev)
        mark_out = torch.empty_like(mark)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.batch_profile):
            ah.copy_bandwidth(0, mark, mark_out)
            ah.solve_batched(bprobs, precision=ah.MIXED, tol=args.tol)
        ah.copy_bandwidth(0, mark, mark_out)
        torch.cuda.synchronize()
        print(f"[bench] {args.batch_profile} mixed batched solves: "
              f"{(time.perf_counter() - t) / args.batch_profile * 1e3:.1f} ms each", file=sys.stderr)
        return
    n = args.n
    t0 = time.perf_counter()
    prob = W.manufactured(W.C3_ALPHA, W.C3_U, (n, n, n), xp="torch", device=dev, chunk=32,
                          with_exact=True)
    u_exact = prob.u_exact
    prob.v_exact = None
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    print(f"[bench] n={n} inputs generated on device in {t_gen:.1f}s", file=sys.stderr, flush=True)

    if args.profile_matvec:
        s = ah.Solver(prob, precision=ah.MIXED if args.profile_prec == "mixed" else ah.FP64)
        q = torch.randn(s.nq, dtype=torch.float64, device=dev)
        for _ in range(args.profile_matvec):
            q = s.schur_apply(q)
            q = q / q.norm()
        torch.cuda.synchronize()
        s.close()
        print(f"[bench] {args.profile_matvec} Schur matvecs done (n={n}, {args.profile_prec})", file=sys.stderr)
        return

    if args.profile_solve:
        s = ah.Solver(prob, precision=ah.MIXED if args.profile_prec == "mixed" else ah.FP64, tol=args.tol)
        out = torch.empty(s.nodal_shape, dtype=torch.float64, device=dev)
        for i in range(2):
            torch.cuda.synchronize()
            time.sleep(0.3)
            t = time.perf_counter()
            _, _, _, st = s.solve(out=out)
            torch.cuda.synchronize()
            print(f"[bench] solve {i} ({args.profile_prec}): {(time.perf_counter() - t) * 1e3:.1f} ms, "
                  f"{st.gmres_iters} GMRES iterations", file=sys.stderr, flush=True)
        s.close()
        return

    # kernel classes that launch kernels themselves (the matvec and residual classes wrap them)
    leaf = ("dst_rows", "dst_strided", "dst_fused", "lift", "rhs_u", "gather", "krylov", "dst_gen",
            "face_reduce", "precond")

    choices = {}

    setup_ms = {}

    def run(prec, steps, warmup, **opts):
        torch.cuda.synchronize()
        t_s = time.perf_counter()
        s = ah.Solver(prob, precision=prec, **opts)
        torch.cuda.synchronize()
        setup_ms["mixed" if prec == ah.MIXED else "fp64"] = (time.perf_counter() - t_s) * 1e3
        # setup-time kernel choice of the operator's plain DST passes (x rows, y strided)
        for name, axis, kind in (("x_rows", 0, 0), ("y_strided", 1, 1)):
            m, tile, td, tg, tb = s.dst_choice(prec, axis, kind)
            choices[f"{'mixed' if prec == ah.MIXED else 'fp64'}_{name}"] = {
                "method": {0: "fft_default", 1: "matrix_core", 2: f"fft_one_tile_{tile}"}.get(
                    m, "fft_default_untimed (no other candidate on arrays of 256 MB or more)"),
                "us_default": td, "us_chosen": tb}
        out = torch.empty(s.nodal_shape, dtype=torch.float64, device=dev)
        for i in range(warmup):
            _, _, _, st = s.solve(out=out)
            print(f"[bench] warmup prec={prec} {st}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        stats = []
        for i in range(steps):
            _, _, _, st = s.solve(out=out)
            stats.append(st)
            print(f"[bench] step prec={prec} {st}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        # one more, untimed and profiled solve: algorithmic bytes of every kernel launched
        s.profile(True)
        s.solve(out=out)
        kt = s.kernel_times()
        model_bytes = sum(c * b for k, (ms, c, b) in kt.items() if k in leaf)
        s.close()
        return out, dt, stats, model_bytes

    # untimed FP64 reference at a tight tolerance: the accuracy yardstick of both forms
    ref = ah.Solver(prob, precision=ah.FP64, tol=1e-13)
    u_ref, _, _, st_ref = ref.solve()
    ref.close()
    print(f"[bench] FP64 reference (tol 1e-13): {st_ref}", file=sys.stderr, flush=True)
    nrm_ref = u_ref.abs().max().item()
    nrm_exact = u_exact.abs().max().item()

    def errs(u):
        return (((u - u_ref).abs().max() / nrm_ref).item(), ((u - u_exact).abs().max() / nrm_exact).item())

    u_mx, dt_mx, st_mx, bytes_mx = run(ah.MIXED, args.steps, args.warmup, tol=args.tol)
    err_mx_ref, err_mx_exact = errs(u_mx)
    del u_mx
    result_fp64 = None
    if not args.no_fp64:
        u_64, dt_64, st_64, bytes_64 = run(ah.FP64, args.steps, args.warmup, tol=args.tol)
        e64_ref, e64_exact = errs(u_64)
        result_fp64 = {"ms_per_step": dt_64 * 1e3, "dof_per_s": n ** 3 / dt_64,
                       "gmres_iters": st_64[-1].gmres_iters, "rel_err_vs_fp64_ref": e64_ref,
                       "rel_err_vs_exact": e64_exact, "speedup_mixed_over_fp64": dt_64 / dt_mx,
                       "model_bytes": bytes_64, "end_to_end_hbm_frac": bytes_64 / dt_64 / (HBM_PEAK_GBS * 1e9)}
        del u_64

    # roofline of the dominant kernel of the FP32 matvec, timed live with HIP events on the
    # solve stream over a few matvecs
    s = ah.Solver(prob, precision=ah.MIXED)
    q = torch.randn(s.nq, dtype=torch.float64, device=dev)
    y = s.schur_apply(q)
    s.profile(True)
    nmv = 4
    for _ in range(nmv):
        y = s.schur_apply(q)
    kt = s.kernel_times()
    s.close()
    del y, q
    ms, cnt, bytes_launch = kt["dst_strided"]
    # reference device bandwidth: the library's calibration copies of a volume of the work
    # arrays' shape (read + write, HIP events): linear, and with the strided y pass's access
    # pattern (its roofline on this device)
    gb = _pattern_copies(ah, torch, dev, n)
    copy_gbps, pattern_gbps = gb["linear"], gb["y_tiles"]
    avg_s = ms / cnt / 1e3
    achieved = bytes_launch / avg_s / 1e9
    pmc = _pmc_traffic(_src_hash())
    traffic = None
    if pmc and pmc["n"] == n:
        traffic = pmc["fetch_bytes"] + pmc["write_bytes"]
    kernels = {k: {"avg_us": (v[0] / v[1] * 1e3 if v[1] else None), "launches_per_matvec": v[1] / nmv,
                   "GBps": (v[2] / (v[0] / v[1] / 1e3) / 1e9 if v[1] and v[0] > 0 else None)}
               for k, v in kt.items() if v[1]}

    # batched form: the 512-instance uneven 2-D workload, whole batch per step, both forms to
    # the same tolerance, errors against a tight FP64 batch solve
    batched = None
    if not args.no_batch:
        specs = W.config4_specs(args.batch_count)
        bprobs = [W.config4_instance(sp, xp="torch", device=dev, with_exact=False) for sp in specs]
        bdof = sum(sp["n"] ** 2 for sp in specs)
        ref_b, _, _ = ah.solve_batched(bprobs, tol=1e-13)
        bres = {}
        for name, prec in (("mixed", ah.MIXED), ("fp64", ah.FP64)):
            ah.solve_batched(bprobs, precision=prec, tol=args.tol)  # warm-up
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                outs, bst, rcb = ah.solve_batched(bprobs, precision=prec, tol=args.tol)
            torch.cuda.synchronize()
            dtb = (time.perf_counter() - t) / args.steps
            err = max(((o - r).abs().max() / r.abs().max()).item() for o, r in zip(outs, ref_b))
            gemm = {}
            for sp, x in zip(specs, bst):
                gemm[sp["n"]] = x.dst_gemm
            bres[name] = {"ms_per_batch": dtb * 1e3, "dof_per_s": bdof / dtb, "max_rel_err_vs_fp64_ref": err,
                          "mean_gmres_iters": sum(x.gmres_iters for x in bst) / len(bst),
                          "all_converged": all(x.converged for x in bst),
                          "matrix_core_dst_by_n": {str(k): bool(v & 1) for k, v in sorted(gemm.items())}}
            print(f"[bench] batched {name}: {dtb*1e3:.1f} ms per batch of {len(bprobs)}", file=sys.stderr, flush=True)
        # the same batch with the FFT kernels only (no setup-time matrix-core choice)
        ah.set_dst_variant(5)
        try:
            ah.solve_batched(bprobs, precision=ah.MIXED, tol=args.tol)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                ah.solve_batched(bprobs, precision=ah.MIXED, tol=args.tol)
            torch.cuda.synchronize()
            bres["mixed_fft_only_ms_per_batch"] = (time.perf_counter() - t) / args.steps * 1e3
        finally:
            ah.set_dst_variant(0)
        # per-instance FP64 loop: one handle and one solve per instance, one after another
        # (setup included, as in the batched call)
        if not args.no_instance_loop:
            torch.cuda.synchronize()
            t = time.perf_counter()
            for pb in bprobs:
                with ah.Solver(pb, precision=ah.FP64, tol=args.tol) as s1:
                    s1.solve()
            torch.cuda.synchronize()
            bres["fp64_instance_loop_ms"] = (time.perf_counter() - t) * 1e3
            print(f"[bench] per-instance FP64 loop: {bres['fp64_instance_loop_ms']:.1f} ms", file=sys.stderr,
                  flush=True)
        batched = {"workload": f"{len(bprobs)} uneven 2-D instances n in {{64..512}} (alpha=1+c sin(2pi p x)cos(2pi q y), "
                               f"u=sin^2 sin^2 cos(k(x+y)), seeded draws), DOF {bdof}",
                   **bres, "speedup_mixed_over_fp64": bres["fp64"]["ms_per_batch"] / bres["mixed"]["ms_per_batch"]}
        if "fp64_instance_loop_ms" in bres:
            batched["speedup_mixed_over_instance_loop"] = bres["fp64_instance_loop_ms"] / bres["mixed"]["ms_per_batch"]
        del bprobs, ref_b

    cpu = None
    same = None
    same2 = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_n, args.tol)
        same = gpu_same_config(ah, W, torch, dev, args.cpu_n, args.tol)
        same["cpu_oracle_s"] = cpu["time_s"]
        same["gpu_mixed_speedup_over_cpu_oracle"] = cpu["time_s"] * 1e3 / same["mixed"]["ms"]
        print(f"[bench] CPU oracle n={args.cpu_n}: {cpu['time_s']:.1f} s; GPU mixed {same['mixed']['ms']:.1f} ms, "
              f"FP64 {same['fp64']['ms']:.1f} ms", file=sys.stderr, flush=True)
        # a second configuration both sides report: the 2-D variable-coefficient problem
        cpu2 = cpu_baseline(args.cpu_n2d, args.tol, dim=2)
        same2 = gpu_same_config(ah, W, torch, dev, args.cpu_n2d, args.tol, dim=2)
        same2["cpu_oracle_s"] = cpu2["time_s"]
        same2["cpu_oracle_sample"] = cpu2["sample"]
        same2["gpu_mixed_speedup_over_cpu_oracle"] = cpu2["time_s"] * 1e3 / same2["mixed"]["ms"]
        print(f"[bench] CPU oracle 2-D n={args.cpu_n2d}: {cpu2['time_s']:.1f} s; GPU mixed {same2['mixed']['ms']:.1f} "
              f"ms, FP64 {same2['fp64']['ms']:.1f} ms", file=sys.stderr, flush=True)

    st = st_mx[-1]
    line = {
        "metric": METRIC,
        "value": n ** 3 / dt_mx,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_mx * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"3-D clamped variable-coefficient biharmonic, n={n}^3, alpha=1+0.5 sin(2pi x)"
                               f"sin(2pi y)sin(2pi z), u=sin^2(pi x)sin^2(pi y)sin^2(pi z); mixed precision "
                               f"(FP32 transforms and stencils inside FP64 refinement on the Schur system), "
                               f"boundary-symbol-preconditioned GMRES(30), Schur tol {args.tol:g}",
                   "n": n, "dof": n ** 3, "interior_dof": (n - 1) ** 3,
                   "gmres_iters": st.gmres_iters, "sweeps": st.sweeps, "schur_relres": st.schur_relres,
                   "rel_err_vs_fp64_ref": err_mx_ref, "rel_err_vs_exact": err_mx_exact,
                   "model_bytes": bytes_mx, "end_to_end_hbm_frac": bytes_mx / dt_mx / (HBM_PEAK_GBS * 1e9),
                   "setup_ms": setup_ms,
                   "time_to_solution_incl_setup_ms": {k: v + (dt_mx * 1e3 if k == "mixed" else
                                                              (result_fp64["ms_per_step"] if result_fp64 else 0.0))
                                                      for k, v in setup_ms.items()},
                   "gpu_same_config": same,
                   "gpu_same_config_2d": same2,
                   "fp64_ref": {"tol": 1e-13, "gmres_iters": st_ref.gmres_iters},
                   "fp64": result_fp64, "batched": batched, "fp32_matvec_kernels": kernels,
                   "dst_kernel_choice": choices},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"k_dst_pipe<float,{n},16,0> (FP32 DST-I pass along y, strided pencils, persistent and pipelined)",
                     "bytes_per_launch": bytes_launch, "avg_launch_us": avg_s * 1e6,
                     "copy_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps,
                     "pattern_copy_GBps": pattern_gbps, "frac_of_pattern_copy": achieved / pattern_gbps,
                     "z_pattern_copy_GBps": gb["z_tiles"]},
        "cpu_baseline": ({k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")} if cpu else None),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
