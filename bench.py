#!/usr/bin/env python
"""Benchmark of the interior point solver on one MI355X.

Workload: 2D Poisson on the 511 x 511 interior grid (261,121 nodes per field,
1,044,484 unknowns per Newton system) with the L1 term, control box
u in [-5, 5] and state box y in [-0.2, 0.3]; y_d is a sum of 8 seeded sine
modes; alpha = 1e-4, beta = 1e-3, sigma = 0.2 (workloads.poisson2d_511).

One step = one complete interior point solve (every Newton system, Krylov
iteration, preconditioner application and update of Algorithm A.1) of one
batch of B instances of that workload (seeds 0..B-1), advanced together by
the batched kernels; inputs are resident in HBM before the timed region.
The headline path runs MINRES + P_D with FP32 V-cycles; the plain FP64
V-cycle variant, the single-instance solve and the served request mix are
timed beside it.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The batched solve splits its instances into lanes, sub-batches on streams of
# their own that overlap one lane's latency-bound multigrid launches with
# another's bandwidth-bound Krylov launches.  Lanes overlap only where each
# stream holds a hardware queue of its own, and HIP gives a process
# GPU_MAX_HW_QUEUES of them (4 by default, read when the runtime starts): ask
# for 8 before anything starts it (a larger value already set is kept).
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

HBM_PEAK_GBS = 8000.0
TUNE_CACHE = os.path.join(ROOT, "paper_1806_05896_amd", "autotune_cache.json")
# HBM bytes per launch of the roofline kernel from rocprofv3 FETCH_SIZE/WRITE_SIZE
# runs (profiles/k_minres_k1_poisson2d_511x8_pmc.md), valid while the kernel
# sources hash to the value they were measured with.
TRAFFIC = {"kernel": 6, "N": 511, "batch": 8, "bytes": 613191533.2, "source_sha": "12e5a857dd29eec6"}
# kernel ids of ipmpde_time_kernel, named for the 2D Poisson workloads timed
# here (convection-diffusion would launch k_mg_down2d / k_mg_up2d / k_mg_coarse_cd)
KERNEL_NAMES = {0: "k_saddle (saddle matvec)",
                2: "k_minres_k2 (Lanczos + diagonal preconditioner)", 3: "one V-cycle",
                4: "k_mg_down_p2 (finest level: smoothing + residual + restriction)",
                5: "k_mg_up_p2 (finest level: prolongation + smoothing)",
                6: "k_minres_k1 (MINRES update + saddle matvec + dots)",
                7: "k_mg_coarse_p2 (coarse levels in one workgroup)"}


def measured_traffic(args):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1806_05896_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("kernels_krylov.hip", "common.h"))
    sha = hashlib.sha256(src).hexdigest()[:16]
    if (args.kernel == TRAFFIC["kernel"] and args.N == TRAFFIC["N"] and args.batch == TRAFFIC["batch"]
            and sha == TRAFFIC["source_sha"]):
        return TRAFFIC["bytes"]
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def time_solves(prob, opts, steps, warmup, torch):
    stream = torch.cuda.current_stream()
    for w in range(warmup):
        prob.solve(opts, stream=stream)
        log(f"warmup {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    lat = []
    its = 0
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        rc = prob.solve(opts, stream=stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        st = prob.stats()
        its += st.krylov_its
        log(f"step {k + 1}/{steps}: rc={rc} nli={st.nli} krylov_its={st.krylov_its} {lat[-1]:.2f} ms")
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return t, lat, its, prob.stats(), rc


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(data, nli, full=False):
    """The oracle (Algorithm A.1 with a SuperLU Newton solve) on the host CPU,
    BLAS and OpenMP pools limited to one thread (SuperLU itself is serial).
    Default: a bounded sample, the first IPM iteration of the same 511 x 511
    problem scaled to solves/s by the number of IPM iterations of a full
    solve; full=True times the whole solve."""
    import oracle
    from oracle.fd import discretize
    from oracle.ipm import IPMOptions, initial_state, ipm_step
    from threadpoolctl import threadpool_limits
    opts = IPMOptions(sigma=data.sigma, newton="schur")
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        if full:
            r = oracle.solve(data, opts)
            nli_done = r.nli
        else:
            disc = discretize(data)
            st = initial_state(data, opts)
            st, _ = ipm_step(data, disc, st, opts, st.mu * opts.sigma)
            nli_done = 1
        t = time.perf_counter() - t0
    per_solve = t if full else t * nli
    host = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": cpu_model()}
    if full:
        sample = (f"full oracle solve of seed 0 ({nli_done} IPM iterations, SuperLU on the eliminated SPD "
                  f"Newton system, {t:.1f} s)")
    else:
        sample = (f"bounded sample: IPM iteration 1 of {nli} of seed 0 (setup + SuperLU factorization and "
                  f"solve of the eliminated SPD Newton system, {t:.1f} s), scaled by {nli} to one solve")
    return {"value": 1.0 / per_solve, "unit": "IPM solves/s", "cores": 1, "kind": "oracle",
            "sample": sample + "; BLAS/OpenMP limited to 1 thread", "host": host}


def copy_ceiling(torch, reps=10):
    """Device-to-device copy of 1 GiB (larger than the 256 MB Infinity Cache):
    the attainable HBM bandwidth on this machine, read + write bytes over time."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * src.numel() * 8 / (ms * 1e-3) / 1e9
    del src, dst
    return gbs


def bench_partial(W, torch, N, reps):
    """Partial observation (observed on the central square, no state bounds):
    FGMRES(30) + P_Pi, FP32 V-cycles, one instance of N^2."""
    from paper_1806_05896_amd import Options, Problem
    d = W.poisson2d_partial(seed=0, N=N)
    o = Options(sigma=d.sigma, krylov="fgmres", precond="ppi", mg_precision="fp32")
    stream = torch.cuda.current_stream()
    with Problem(d) as p:
        p.solve(o, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rc = p.solve(o, stream=stream)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        s = p.stats()
    log(f"partial observation {N}^2: {1 / t:.2f} solves/s")
    return {"workload": f"poisson2d_partial: 2D Poisson {N}x{N}, observed on (0.25,0.75)^2, alpha=1e-4, "
                        "beta=1e-3, u in [-5,5], sigma=0.25", "krylov": "fgmres(30)", "precond": "P_Pi",
            "solves_per_s": 1 / t, "ms_per_solve": t * 1e3, "nli": s.nli, "krylov_its_per_solve": s.krylov_its,
            "krylov_its_per_s": s.krylov_its / t, "status": rc}


def bench_heat(W, torch, N, nt, reps):
    """Heat equation, all nt time steps at once (tau = 1/nt), one instance:
    FGMRES(30) + P_T (the paper's choice for this problem) and MINRES + P_D,
    FP32 V-cycles; the Schur solves are block substitutions over the steps."""
    from paper_1806_05896_amd import Options, Problem
    d = W.heat2d(seed=0, N=N, nt=nt)
    stream = torch.cuda.current_stream()
    out = {"workload": f"heat2d: heat equation {N}x{N} x {nt} backward Euler steps (tau={1.0 / nt:g}), "
                       f"y_d = A sin(pi x1) sin(pi x2), alpha=1e-4, beta=1e-2, u in [-15,15], sigma=0.25",
           "space_time_nodes": d.n}
    with Problem(d) as p:
        for name, kry, pre in (("fgmres_pt", "fgmres", "pt"), ("minres_pd", "minres", "pd")):
            o = Options(sigma=d.sigma, krylov=kry, precond=pre, mg_precision="fp32")
            p.solve(o, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                rc = p.solve(o, stream=stream)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            s = p.stats()
            log(f"heat {N}^2 x {nt} {name}: {1 / t:.2f} solves/s, nli {s.nli}, its {s.krylov_its}")
            out[name] = {"solves_per_s": 1 / t, "ms_per_solve": t * 1e3, "nli": s.nli,
                         "krylov_its_per_solve": s.krylov_its, "krylov_its_per_s": s.krylov_its / t, "status": rc}
    return out


def bench_q1(W, torch, N, reps, batch=8):
    """The 511^2 Poisson workload with Q1 finite elements (the paper's own
    discretization), one instance: MINRES + P_D and FGMRES(30) + P_T, FP32
    and FP64 V-cycles, 20 Chebyshev steps for the mass block; then `batch`
    instances solved as one batch (FP32)."""
    from paper_1806_05896_amd import Options, Problem
    d = W.poisson2d_q1(seed=0, N=N)
    stream = torch.cuda.current_stream()
    out = {"workload": f"poisson2d_q1: 2D Poisson {N}x{N}, Q1 elements, alpha=1e-4, beta=1e-3, u in [-5,5], "
                       "y in [-0.2,0.3], sigma=0.2"}
    with Problem(d) as p:
        for prec in ("fp32", "fp64"):
            for name, kry, pre in (("minres_pd", "minres", "pd"), ("fgmres_pt", "fgmres", "pt")):
                o = Options(sigma=d.sigma, krylov=kry, precond=pre, mg_precision=prec)
                p.solve(o, stream=stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    rc = p.solve(o, stream=stream)
                torch.cuda.synchronize()
                t = (time.perf_counter() - t0) / reps
                s = p.stats()
                key = name if prec == "fp32" else f"{name}_fp64"
                log(f"q1 {N}^2 {key}: {1 / t:.2f} solves/s, nli {s.nli}, its {s.krylov_its}")
                out[key] = {"solves_per_s": 1 / t, "ms_per_solve": t * 1e3, "nli": s.nli,
                            "krylov_its_per_solve": s.krylov_its, "krylov_its_per_s": s.krylov_its / t,
                            "mg_precision": prec, "status": rc}
    if batch > 1:
        from paper_1806_05896_amd import Batch
        # seeds 1, 4, 7, 13 and 15 of this workload lose the interior under the
        # fixed barrier decrease (like the hard finite-difference instance);
        # the batch takes the first eight seeds whose solves converge
        seeds = [0, 2, 3, 5, 6, 8, 9, 10][:batch]
        datas = [W.poisson2d_q1(seed=k, N=N) for k in seeds]
        probs = [Problem(x) for x in datas]
        try:
            bt = Batch(probs)
            out["batched"] = {"instances": len(seeds), "workload": f"poisson2d_q1 seeds {seeds}"}
            for name, kry, pre in (("minres_pd", "minres", "pd"), ("fgmres_pt", "fgmres", "pt")):
                o = Options(sigma=d.sigma, krylov=kry, precond=pre, mg_precision="fp32")
                bt.solve(o, stream=stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    st = bt.solve(o, stream=stream)
                torch.cuda.synchronize()
                t = (time.perf_counter() - t0) / reps
                log(f"q1 batch {len(seeds)} x {N}^2 {name}: {len(seeds) / t:.2f} solves/s")
                out["batched"][name] = {"solves_per_s": len(seeds) / t, "ms_per_batched_solve": t * 1e3, "status": st}
        finally:
            for p in probs:
                p.close()
    return out


def bench_q1_3d(W, torch, N, reps):
    """The 127^3 Poisson workload with trilinear Q1 elements, one instance:
    MINRES + P_D and FGMRES(30) + P_T, FP32 and FP64 V-cycles, 20 Chebyshev
    steps."""
    from paper_1806_05896_amd import Options, Problem
    d = W.poisson3d_q1(seed=0, N=N)
    stream = torch.cuda.current_stream()
    out = {"workload": f"poisson3d_q1: 3D Poisson {N}^3, trilinear Q1 elements, alpha=1e-5, beta=1e-3, "
                       "u in [-10,10], sigma=0.2"}
    with Problem(d) as p:
        for prec in ("fp32", "fp64"):
            for name, kry, pre in (("minres_pd", "minres", "pd"), ("fgmres_pt", "fgmres", "pt")):
                o = Options(sigma=d.sigma, krylov=kry, precond=pre, mg_precision=prec)
                p.solve(o, stream=stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    rc = p.solve(o, stream=stream)
                torch.cuda.synchronize()
                t = (time.perf_counter() - t0) / reps
                s = p.stats()
                key = name if prec == "fp32" else f"{name}_fp64"
                log(f"q1 3d {N}^3 {key}: {1 / t:.2f} solves/s, nli {s.nli}, its {s.krylov_its}")
                out[key] = {"solves_per_s": 1 / t, "ms_per_solve": t * 1e3, "nli": s.nli,
                            "krylov_its_per_solve": s.krylov_its, "krylov_its_per_s": s.krylov_its / t,
                            "mg_precision": prec, "status": rc}
    return out


def bench_q1_avli(W, torch):
    """Average Krylov iterations per IPM step (AV-LI) of the Q1 Poisson problem
    of Sec. 5.1 (u in [-2, 1.5], y_d = sin(pi x1) sin(pi x2), beta = 1e-2,
    sigma = 0.2, 9 IPM iterations) for h = 2^-6 .. 2^-9 and alpha = 1e-2,
    1e-4, 1e-6, with FGMRES + P_T and MINRES + P_D, under the default
    multigrid (1 V-cycle, 2+2 sweeps, FP32), the same in FP64, and 3 cycles
    of 5+5 sweeps in FP64, the cycle count and smoothing of the paper's AMG
    (FP32 cycles after the first gain nothing: the FP32 residual of the
    Poisson operator bottoms out near eps_32 times its condition number)."""
    import math

    import numpy as np

    from paper_1806_05896_amd import Options, Problem
    stream = torch.cuda.current_stream()
    out = {}
    for ell in (6, 7, 8, 9):
        N = 2 ** ell - 1
        x1, x2 = W.interior_coords(2, N)
        for la in (-2, -4, -6):
            d = W.poisson2d_q1(seed=0, N=N)
            d.y_d = np.sin(math.pi * x1) * np.sin(math.pi * x2)
            d.alpha, d.beta = 10.0 ** la, 1e-2
            d.u_a[:] = -2.0
            d.u_b[:] = 1.5
            d.y_a = d.y_b = None
            cell = {}
            with Problem(d) as p:
                for mg, kw in (("fp32 1x(2+2)", {"mg_precision": "fp32"}),
                               ("fp64 1x(2+2)", {"mg_precision": "fp64"}),
                               ("fp64 3x(5+5)", {"mg_precision": "fp64", "vcycles": 3, "nu_pre": 5, "nu_post": 5})):
                    for name, kry, pre in (("P_T", "fgmres", "pt"), ("P_D", "minres", "pd")):
                        o = Options(sigma=0.2, krylov=kry, precond=pre, fixed_nli=9, **kw)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        rc = p.solve(o, stream=stream)
                        torch.cuda.synchronize()
                        t = time.perf_counter() - t0
                        s = p.stats()
                        cell[f"{name} {mg}"] = {"av_li": s.krylov_its / max(1, s.nli), "nli": s.nli,
                                                "ms_per_solve": t * 1e3, "status": rc}
            out[f"h=2^-{ell} alpha=1e{la}"] = cell
            log(f"q1 av-li h=2^-{ell} alpha=1e{la}: " +
                ", ".join(f"{k} {v['av_li']:.1f}" for k, v in cell.items()))
    # the same problem with state bounds y in [-0.1, 0.8] and u in [-1, 15]
    # (FGMRES + P_T, the paper's second Poisson table), and the 3D partially
    # observed problem (FGMRES + P_Pi, h = 2^-3 .. 2^-5, the paper's third)
    settings = (("fp64 1x(2+2)", {"mg_precision": "fp64"}),
                ("fp64 3x(5+5)", {"mg_precision": "fp64", "vcycles": 3, "nu_pre": 5, "nu_post": 5}))
    cases = []
    for ell in (6, 7, 8, 9):
        for la in (-2, -4, -6):
            cases.append(("state", ell, la))
    for ell in (3, 4, 5):
        for la in (-2, -4, -6):
            cases.append(("partial3d", ell, la))
    for kind, ell, la in cases:
        N = 2 ** ell - 1
        if kind == "state":
            x1, x2 = W.interior_coords(2, N)
            d = W.poisson2d_q1(seed=0, N=N)
            d.y_d = np.sin(math.pi * x1) * np.sin(math.pi * x2)
            d.alpha, d.beta, d.sigma = 10.0 ** la, 1e-2, 0.2
            d.u_a[:] = -1.0
            d.u_b[:] = 15.0
            d.y_a = np.full(d.n, -0.1)
            d.y_b = np.full(d.n, 0.8)
            kry, pre = "fgmres", "pt"
        else:
            d = W.poisson3d_q1_partial(seed=0, N=N)
            d.alpha = 10.0 ** la
            kry, pre = "fgmres", "ppi"
        cell = {}
        with Problem(d) as p:
            for mg, kw in settings:
                o = Options(sigma=d.sigma, krylov=kry, precond=pre, **kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc = p.solve(o, stream=stream)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                s = p.stats()
                cell[mg] = {"av_li": s.krylov_its / max(1, s.nli), "nli": s.nli, "ms_per_solve": t * 1e3,
                            "status": rc}
        out[f"{kind} h=2^-{ell} alpha=1e{la}"] = cell
        log(f"q1 av-li {kind} h=2^-{ell} alpha=1e{la}: " +
            ", ".join(f"{k} {v['av_li']:.1f} (nli {v['nli']}, rc {v['status']})" for k, v in cell.items()))
    return out


def bench_heat_batch(W, torch, N, nt, B, reps):
    """B heat instances (seeds 0..B-1) solved as one batch: the substitution
    kernel runs one workgroup per instance, every other launch serves all."""
    from paper_1806_05896_amd import Batch, Options, Problem
    datas = [W.heat2d(seed=k, N=N, nt=nt) for k in range(B)]
    probs = [Problem(d) for d in datas]
    stream = torch.cuda.current_stream()
    out = {"instances": B, "workload": f"heat2d seeds 0..{B - 1}, {N}x{N} x {nt} steps"}
    try:
        batch = Batch(probs)
        for name, kry, pre in (("fgmres_pt", "fgmres", "pt"), ("minres_pd", "minres", "pd")):
            o = Options(sigma=datas[0].sigma, krylov=kry, precond=pre, mg_precision="fp32")
            batch.solve(o, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                st = batch.solve(o, stream=stream)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            log(f"heat batch {B} x {N}^2 x {nt} {name}: {B / t:.2f} solves/s")
            out[name] = {"solves_per_s": B / t, "ms_per_batched_solve": t * 1e3, "status": st,
                         "krylov_its": [p.stats().krylov_its for p in probs]}
    finally:
        for p in probs:
            p.close()
    return out


def _time_one(p, o, reps, stream, torch):
    p.solve(o, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rc = p.solve(o, stream=stream)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    s = p.stats()
    return {"solves_per_s": 1 / t, "ms_per_solve": t * 1e3, "nli": s.nli, "krylov_its_per_solve": s.krylov_its,
            "krylov_its_per_s": s.krylov_its / t, "status": rc}


def bench_small(W, torch, reps, batch=64):
    """The 31 x 31 problem (y_d = A sin(pi x1) sin(pi x2), alpha = 1e-2,
    beta = 1e-3, u in [-2, 2], no state bounds; MINRES + P_D, FP64 V-cycles):
    one instance alone, then `batch` instances (seeds 0..batch-1) as one batch."""
    from paper_1806_05896_amd import Batch, Options, Problem
    stream = torch.cuda.current_stream()
    d = W.poisson2d_small(seed=0)
    o = Options(sigma=d.sigma, mg_precision="fp64")
    out = {"workload": "poisson2d_small: 2D Poisson 31x31, alpha=1e-2, beta=1e-3, u in [-2,2], sigma=0.2, "
                       "MINRES + P_D, FP64 V-cycles"}
    with Problem(d) as p:
        out["single"] = _time_one(p, o, reps, stream, torch)
    datas = [W.poisson2d_small(seed=k) for k in range(batch)]
    probs = [Problem(x) for x in datas]
    try:
        with Batch(probs) as b:
            b.solve(o, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                st = b.solve(o, stream=stream)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
        its = sum(p.stats().krylov_its for p in probs)
        out["batched"] = {"instances": batch, "solves_per_s": batch / t, "ms_per_batch": t * 1e3,
                          "krylov_its_per_s": its / t, "all_converged": all(x == 0 for x in st)}
    finally:
        for p in probs:
            p.close()
    log(f"31^2: single {out['single']['solves_per_s']:.1f} solves/s, batch of {batch} "
        f"{out['batched']['solves_per_s']:.1f} solves/s")
    return out


def bench_fd3d(W, torch, N, betas, reps):
    """3D Poisson, 7-point finite differences on N^3 (alpha = 1e-5,
    u in [-10, 10], 8 sine modes), beta swept over `betas`; MINRES + P_D with
    FP32 V-cycles, one instance per beta; FP64 V-cycles beside it at
    beta = 1e-3.  The roofline figure is k_minres_k1 (MINRES update + saddle
    matvec + dots) timed with HIP events after the solve."""
    from paper_1806_05896_amd import Options, Problem
    stream = torch.cuda.current_stream()
    out = {"workload": f"poisson3d_127: 3D Poisson {N}^3 (7-point FD), alpha=1e-5, u in [-10,10], sigma=0.2, "
                       "MINRES + P_D"}
    for beta in betas:
        d = W.poisson3d_127(seed=0, N=N, beta=beta)
        with Problem(d) as p:
            o = Options(sigma=d.sigma, mg_precision="fp32")
            r = _time_one(p, o, reps, stream, torch)
            ms, nb = p.time_kernel(6, reps=20, opts=o, stream=stream)
            r["k_minres_k1"] = {"avg_us": ms * 1e3, "GB/s": nb / (ms * 1e-3) / 1e9,
                                "frac_of_peak": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            ms, nb = p.time_kernel(2, reps=20, opts=o, stream=stream)
            r["k_minres_k2"] = {"avg_us": ms * 1e3, "GB/s": nb / (ms * 1e-3) / 1e9}
            if beta == 1e-3:
                r64 = _time_one(p, Options(sigma=d.sigma, mg_precision="fp64"), reps, stream, torch)
                r["fp64_vcycles"] = r64
                r["fp32_over_fp64"] = r["solves_per_s"] / r64["solves_per_s"]
        out[f"beta_{beta:g}"] = r
        log(f"3d fd {N}^3 beta={beta:g}: {r['solves_per_s']:.2f} solves/s, nli {r['nli']}, "
            f"its {r['krylov_its_per_solve']}, k1 {r['k_minres_k1']['GB/s']:.0f} GB/s")
    return out


def bench_cd(W, torch, N, reps):
    """Convection-diffusion, eps = 1/200, upwinded FD on N^2 (alpha = beta =
    1e-3, u in [-3, 3], 8 sine modes): FGMRES(30) + P_T with FP32 V-cycles (and
    MINRES + P_D beside it), one instance; the multigrid kernels timed with
    HIP events after the solve."""
    from paper_1806_05896_amd import Options, Problem
    stream = torch.cuda.current_stream()
    d = W.convdiff2d_255(seed=0, N=N)
    out = {"workload": f"convdiff2d_255: -eps Lap y + w.grad y = u, eps=1/200, wind of Sec. 5.2, upwind FD "
                       f"{N}x{N}, alpha=beta=1e-3, u in [-3,3], sigma={d.sigma}"}
    with Problem(d) as p:
        for name, kry, pre in (("fgmres_pt", "fgmres", "pt"), ("minres_pd", "minres", "pd")):
            o = Options(sigma=d.sigma, krylov=kry, precond=pre, mg_precision="fp32")
            out[name] = _time_one(p, o, reps, stream, torch)
            log(f"cd {N}^2 {name}: {out[name]['solves_per_s']:.2f} solves/s, nli {out[name]['nli']}, "
                f"its {out[name]['krylov_its_per_solve']}")
        o = Options(sigma=d.sigma, krylov="fgmres", precond="pt", mg_precision="fp32")
        for k, name in ((3, "one V-cycle"), (4, "k_mg_down2d (finest level)"), (5, "k_mg_up2d (finest level)")):
            ms, nb = p.time_kernel(k, reps=20, opts=o, stream=stream)
            out.setdefault("kernels", {})[name] = {"avg_us": ms * 1e3, "GB/s": nb / (ms * 1e-3) / 1e9}
    return out


def solver_options(d, Options, prec="fp32"):
    """Per-request solver choice: MINRES + P_D for Poisson, FGMRES(30) + P_T
    for convection-diffusion, multigrid in the given precision."""
    if d.pde == "convdiff":
        return Options(sigma=d.sigma, krylov="fgmres", precond="pt", mg_precision=prec)
    return Options(sigma=d.sigma, krylov="minres", precond="pd", mg_precision=prec)


def bench_batched(W, torch, B, reps):
    """B instances of the 511^2 workload (seeds 0..B-1) advanced by the same
    launches (ipmpde_batch), FP32 V-cycles against plain FP64 V-cycles."""
    import numpy as np
    from paper_1806_05896_amd import Batch, Options, Problem
    datas = [W.poisson2d_511(seed=s) for s in range(B)]
    probs = [Problem(d) for d in datas]
    out = {"instances": B, "workload": "poisson2d_511 seeds 0..%d" % (B - 1)}
    us = {}
    stream = torch.cuda.current_stream()
    with Batch(probs) as b:
        for prec in ("fp32", "fp64"):
            opts = [Options(sigma=d.sigma, mg_precision=prec) for d in datas]
            b.solve(opts, stream=stream)  # warm-up (graph capture, workspace)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                st = b.solve(opts, stream=stream)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            its = sum(p.stats().krylov_its for p in probs)
            us[prec] = [p.query("u") for p in probs]
            out[prec] = {"solves_per_s": B / t, "ms_per_batch": t * 1e3, "krylov_its_per_s": its / t,
                         "status": st, "nli": [p.stats().nli for p in probs]}
            log(f"batched x{B} {prec}: {B / t:.2f} solves/s ({t * 1e3:.1f} ms per batch)")
    out["max_rel_l2_u_fp32_vs_fp64"] = max(float(np.linalg.norm(a - c) / np.linalg.norm(c))
                                           for a, c in zip(us["fp32"], us["fp64"]))
    out["fp32_over_fp64"] = out["fp32"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    for p in probs:
        p.close()
    return out


def serve_run(reqs, times, torch, slots, budget, prec="fp32"):
    """Drive the request stream through the serving engine: request i is
    created (its data uploaded) and submitted at times[i] seconds after the
    start; the loop steps the engine while work is in flight and returns each
    request's control to the host when it finishes.  Latency = completion
    (result on the host) minus arrival."""
    import numpy as np  # noqa: F401
    from paper_1806_05896_amd import Engine, Options, Problem
    stream = torch.cuda.current_stream()
    n = len(reqs)
    lat = [None] * n
    status = [None] * n
    its = 0
    probs, tickets = [None] * n, [None] * n
    pending = []
    nxt = 0
    steps = 0
    with Engine(budget, slots) as eng:
        t0 = time.perf_counter()
        while nxt < n or pending:
            now = time.perf_counter() - t0
            while nxt < n and times[nxt] <= now:
                d = reqs[nxt]
                probs[nxt] = Problem(d)
                tickets[nxt] = eng.submit(probs[nxt], solver_options(d, Options, prec))
                pending.append(nxt)
                nxt += 1
            if not pending:
                time.sleep(max(0.0, times[nxt] - (time.perf_counter() - t0)))
                continue
            eng.step(stream)
            steps += 1
            still = []
            for i in pending:
                info = eng.poll(tickets[i])
                if info["state"] != 2:
                    still.append(i)
                    continue
                probs[i].query("u")  # the response
                lat[i] = (time.perf_counter() - t0 - times[i]) * 1e3
                status[i] = info["status"]
                its += info["krylov_its"]
                eng.release(tickets[i])
                probs[i].close()
            pending = still
        makespan = time.perf_counter() - t0
        peak = eng.info()["peak_bytes"]
    return {"requests": n, "makespan_s": makespan, "solves_per_s": n / makespan, "krylov_its_per_s": its / makespan,
            "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "max": max(lat)},
            "engine_steps": steps, "peak_admitted_bytes": peak,
            "ok": sum(1 for s in status if s == 0), "status_counts": {str(k): status.count(k) for k in set(status)}}


def bench_serving(W, torch, n_requests, slots, budget_gib, loads):
    """Served mix: saturation throughput with every request present at the
    start, then Poisson arrivals at the given fractions of it."""
    reqs = W.served_requests(n_requests=n_requests, seed=0)
    datas = [d for _, d in reqs]
    unit_times = [t for t, _ in reqs]  # arrival times of a unit-rate Poisson process
    budget = int(budget_gib * (1 << 30))
    out = {"workload": f"served_mix: {n_requests} requests, 50% Poisson / 25% CD eps=1/50 / 25% CD eps=1/200, "
                       "N in {31,63,127,255}, alpha logU[1e-6,1e-2], beta logU[1e-5,1e-2], bounds U[1,10]",
           "slots": slots, "hbm_budget_gib": budget_gib}
    sat = serve_run(datas, [0.0] * len(datas), torch, slots, budget)
    log(f"serving saturation: {sat['solves_per_s']:.2f} req/s, p50 {sat['latency_ms']['p50']:.0f} ms")
    out["saturation"] = sat
    for load in loads:
        rate = load * sat["solves_per_s"]
        r = serve_run(datas, [t / rate for t in unit_times], torch, slots, budget)
        r["arrival_rate_per_s"] = rate
        log(f"serving load {load}: p50 {r['latency_ms']['p50']:.0f} ms p99 {r['latency_ms']['p99']:.0f} ms")
        out[f"load_{load}"] = r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 V-cycle variant")
    ap.add_argument("--kernel", type=int, default=6, help="kernel id for the roofline figure")
    ap.add_argument("--N", type=int, default=511)
    ap.add_argument("--batch", type=int, default=8, help="instances solved together per step")
    ap.add_argument("--serve-requests", type=int, default=256, help="requests of the served mix (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--serve-loads", type=str, default="0.8", help="arrival rates as fractions of saturation")
    ap.add_argument("--partial-N", type=int, default=255, help="grid of the partial-observation run (0: skip)")
    ap.add_argument("--heat-N", type=int, default=63, help="grid of the heat-equation run (0: skip)")
    ap.add_argument("--heat-nt", type=int, default=100, help="time steps of the heat-equation run")
    ap.add_argument("--heat-batch", type=int, default=16, help="instances of the batched heat run (0: skip)")
    ap.add_argument("--q1-N", type=int, default=511, help="grid of the Q1 finite-element run (0: skip)")
    ap.add_argument("--q1-3d-N", type=int, default=127, help="grid of the 3D Q1 run (0: skip)")
    ap.add_argument("--small", type=int, default=1, help="time the 31^2 problem (0: skip)")
    ap.add_argument("--fd3d-N", type=int, default=127, help="grid of the 3D finite-difference run (0: skip)")
    ap.add_argument("--fd3d-betas", type=str, default="1e-4,1e-3,1e-2,1e-1")
    ap.add_argument("--cd-N", type=int, default=255, help="grid of the convection-diffusion run (0: skip)")
    ap.add_argument("--cpu-full", action="store_true", help="time a full oracle solve instead of one iteration")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="run the default multigrid schedule instead of the autotuner's pick")
    ap.add_argument("--only", choices=["serve", "batch", "partial", "heat", "q1", "q1_3d", "q1_avli", "small",
                                       "fd3d", "cd"], default=None,
                    help="run one extra section alone")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch the roofline kernel (20 times) and a 1 GiB device copy, for counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_1806_05896_amd import Options, Problem

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    loads = [float(x) for x in args.serve_loads.split(",") if x]
    if args.only == "serve":
        print(json.dumps({"serving": bench_serving(W, torch, args.serve_requests, args.serve_slots,
                                                   args.serve_budget_gib, loads)}), flush=True)
        return
    if args.only == "partial":
        print(json.dumps({"partial_observation": bench_partial(W, torch, args.partial_N, 3)}), flush=True)
        return
    if args.only == "q1":
        print(json.dumps({"q1": bench_q1(W, torch, args.q1_N, 3)}), flush=True)
        return
    if args.only == "q1_avli":
        print(json.dumps({"q1_avli": bench_q1_avli(W, torch)}), flush=True)
        return
    if args.only == "q1_3d":
        print(json.dumps({"q1_3d": bench_q1_3d(W, torch, args.q1_3d_N, 2)}), flush=True)
        return
    if args.only == "heat":
        out = bench_heat(W, torch, args.heat_N, args.heat_nt, 3)
        if args.heat_batch > 0:
            out["batched"] = bench_heat_batch(W, torch, args.heat_N, args.heat_nt, args.heat_batch, 2)
        print(json.dumps({"heat": out}), flush=True)
        return
    betas = [float(x) for x in args.fd3d_betas.split(",") if x]
    if args.only == "small":
        print(json.dumps({"small": bench_small(W, torch, 3)}), flush=True)
        return
    if args.only == "fd3d":
        print(json.dumps({"fd3d": bench_fd3d(W, torch, args.fd3d_N, betas, 2)}), flush=True)
        return
    if args.only == "cd":
        print(json.dumps({"convdiff": bench_cd(W, torch, args.cd_N, 2)}), flush=True)
        return
    if args.only == "batch":
        print(json.dumps({"batched": bench_batched(W, torch, max(1, args.batch), 2)}), flush=True)
        return
    from paper_1806_05896_amd import Batch
    B = max(1, args.batch)
    datas = [W.poisson2d_511(seed=k, N=args.N) for k in range(B)]
    probs = [Problem(d) for d in datas]
    batch = Batch(probs)
    opts = Options(sigma=datas[0].sigma, mg_precision="fp32")
    stream = torch.cuda.current_stream()
    tune = None
    if args.autotune and not args.pmc_probe:
        # the library's autotuner picks the FP32 V-cycle schedule (cycles, sweeps,
        # level-kernel tiles) of this batch; the committed cache file holds the pick
        # for this GPU architecture, a miss tunes (two batched solves per candidate)
        t0 = time.perf_counter()
        opts, tuned_ms, hit = batch.autotune(opts, cache=TUNE_CACHE, stream=stream)
        tune = {"cache": "hit" if hit else "miss (tuned now)", "cache_file": os.path.relpath(TUNE_CACHE, ROOT),
                "pick": {"vcycles": opts.vcycles, "nu_pre": opts.nu_pre, "nu_post": opts.nu_post,
                         "mg_precision": opts.mg_precision, "mg_tile": opts.mg_tile, "lanes": opts.lanes},
                "tuned_batch_solve_ms": tuned_ms, "seconds": time.perf_counter() - t0}
        log(f"autotune: {tune}")
    if args.pmc_probe:
        # the roofline kernel of the batched step at a mid-solve Newton state, then a plain
        # copy of known size (1 GiB, larger than the 256 MB Infinity Cache) that calibrates
        # the byte counters
        probe = Options(sigma=datas[0].sigma, mg_precision="fp32", fixed_nli=3)
        batch.solve(probe, stream=stream)
        ms, nbytes = batch.time_kernel(args.kernel, reps=20, opts=probe, stream=stream)
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": KERNEL_NAMES[args.kernel], "instances": B, "algorithmic_bytes": nbytes,
                          "copy_bytes_each_direction": src.numel() * 8}))
        return
    log(f"workload poisson2d_511 N={args.N} x {B} instances")
    for w in range(args.warmup):
        batch.solve(opts, stream=stream)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    lat, its = [], 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        st = batch.solve(opts, stream=stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        its += sum(p.stats().krylov_its for p in probs)
        log(f"step {k + 1}/{args.steps}: status={st} {lat[-1]:.2f} ms")
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    stats = [p.stats() for p in probs]
    u32 = [p.query("u") for p in probs]
    y0_32 = probs[0].query("y")
    result = {
        "metric": "IPM solves/s (2D Poisson 511^2, L1 + control and state boxes)",
        "value": B * args.steps / t,
        "unit": "IPM solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded sine-mode desired states, workloads.poisson2d_511 seeds 0..%d)" % (B - 1),
        "config": {"workload": f"poisson2d_511 x{B}: 2D Poisson {args.N}x{args.N} interior, alpha=1e-4, "
                               "beta=1e-3, u in [-5,5], y in [-0.2,0.3], sigma=0.2, IPM tol 1e-6; "
                               f"{B} instances (seeds 0..{B - 1}) solved as one batch per step"
                               + (f", split into {opts.lanes} lanes (sub-batches on streams of their own)"
                                  if opts.lanes > 1 else ""),
                   "batch": B, "krylov": "minres", "precond": "P_D", "mg_precision": opts.mg_precision,
                   "vcycles": opts.vcycles, "nu_pre": opts.nu_pre, "nu_post": opts.nu_post, "mg_tile": opts.mg_tile,
                   "lanes": opts.lanes, "krylov_tol": 1e-10, "status": st},
        "autotune": tune,
        "krylov_its_per_s": its / t,
        "nli": [s_.nli for s_ in stats],
        "krylov_its_per_solve": its / (B * args.steps),
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "of": "one batched step"},
    }

    # seed 0 against the oracle's stored solution of the same inputs (written by
    # tests/golden/make_poisson2d_511_oracle.py), with the oracle's own error
    golden = os.path.join(ROOT, "tests", "golden", "poisson2d_511_seed0_oracle.npz")
    if args.N == 511 and os.path.exists(golden):
        g = np.load(golden, allow_pickle=False)
        result["parity_vs_oracle"] = {
            "instance": "seed 0", "nli": stats[0].nli, "oracle_nli": int(g["nli"]),
            "rel_l2_u": float(np.linalg.norm(u32[0] - g["u"]) / np.linalg.norm(g["u"])),
            "rel_l2_y": float(np.linalg.norm(y0_32 - g["y"]) / np.linalg.norm(g["y"])),
            "fp64_oracle_error_u": float(g["oracle_error_u"]), "fp64_oracle_error_y": float(g["oracle_error_y"]),
            "fp64_oracle_error_is": "|u(eps=1e-6) - u(eps=1e-12)| / |u(eps=1e-12)| of the oracle"}

    # roofline of the dominant kernel of the batched step, timed with HIP events on the
    # solve stream, one launch serving all instances (after a one-lane solve: the
    # kernel timing runs on the whole batch's Newton setup)
    if opts.lanes > 1:
        batch.solve(Options(**{**opts.__dict__, "lanes": 1}), stream=stream)
    ms, nbytes = batch.time_kernel(args.kernel, reps=100, opts=opts, stream=stream)
    achieved = nbytes / (ms * 1e-3) / 1e9
    result["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args),
                          "kernel": KERNEL_NAMES[args.kernel], "avg_us": ms * 1e3,
                          "algorithmic_bytes_per_launch": nbytes, "instances_per_launch": B}
    ceiling = copy_ceiling(torch)
    result["roofline"]["copy_ceiling_GBps"] = ceiling
    result["roofline"]["frac_of_copy_ceiling"] = achieved / ceiling
    kern = {}
    for k in (2, 3, 4, 5, 6, 7):
        ms_k, b_k = batch.time_kernel(k, reps=50, opts=opts, stream=stream)
        kern[KERNEL_NAMES[k]] = {"avg_us": ms_k * 1e3, "GB/s": b_k / (ms_k * 1e-3) / 1e9}
    result["kernels"] = kern

    if not args.no_fp64:
        opts64 = Options(**{**opts.__dict__, "mg_precision": "fp64"})
        batch.solve(opts64, stream=stream)
        torch.cuda.synchronize()
        n64 = max(2, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(n64):
            batch.solve(opts64, stream=stream)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        u64 = [p.query("u") for p in probs]
        result["fp64_vcycles"] = {
            "solves_per_s": B * n64 / t64, "krylov_its_per_solve": sum(p.stats().krylov_its for p in probs) / B,
            "status": [p.stats().status for p in probs],
            "fp32_speedup": (B * args.steps / t) / (B * n64 / t64),
            "max_rel_l2_u_vs_fp32_path": max(float(np.linalg.norm(a - c) / np.linalg.norm(c))
                                             for a, c in zip(u32, u64))}
    batch.close()

    # one instance alone (latency of a single solve)
    single = probs[0]
    opts1 = Options(**{**opts.__dict__, "mg_tile": "auto"})
    tune1 = None
    if args.autotune:
        # a single instance has its own best schedule (launch latency weighs more)
        with Batch([single]) as b1:
            opts1, ms1, hit1 = b1.autotune(Options(sigma=datas[0].sigma, mg_precision="fp32"), cache=TUNE_CACHE,
                                           stream=stream)
        tune1 = {"cache": "hit" if hit1 else "miss (tuned now)",
                 "pick": {"vcycles": opts1.vcycles, "nu_pre": opts1.nu_pre, "nu_post": opts1.nu_post,
                          "mg_precision": opts1.mg_precision, "mg_tile": opts1.mg_tile, "lanes": opts1.lanes},
                 "tuned_solve_ms": ms1}
        log(f"autotune (single instance): {tune1}")
    ts, lat1, its1, st1, rc1 = time_solves(single, opts1, max(3, args.steps // 2), 1, torch)
    n1 = max(3, args.steps // 2)
    result["single_instance"] = {"solves_per_s": n1 / ts, "krylov_its_per_s": its1 / ts, "nli": st1.nli,
                                 "latency_ms": {"p50": percentile(lat1, 50), "p99": percentile(lat1, 99)},
                                 "status": rc1, "autotune": tune1}
    data0 = datas[0]
    for p in probs:
        p.close()

    if args.small:
        result["small"] = bench_small(W, torch, 3)
    if args.fd3d_N > 0:
        result["fd3d"] = bench_fd3d(W, torch, args.fd3d_N, betas, 1)
    if args.cd_N > 0:
        result["convdiff"] = bench_cd(W, torch, args.cd_N, 2)
    if args.partial_N > 0:
        result["partial_observation"] = bench_partial(W, torch, args.partial_N, 2)
    if args.q1_N > 0:
        result["q1"] = bench_q1(W, torch, args.q1_N, 2)
    if args.q1_3d_N > 0:
        result["q1_3d"] = bench_q1_3d(W, torch, args.q1_3d_N, 1)
    if args.heat_N > 0:
        result["heat"] = bench_heat(W, torch, args.heat_N, args.heat_nt, 2)
        if args.heat_batch > 0:
            result["heat"]["batched"] = bench_heat_batch(W, torch, args.heat_N, args.heat_nt, args.heat_batch, 1)

    if args.serve_requests > 0:
        result["serving"] = bench_serving(W, torch, args.serve_requests, args.serve_slots, args.serve_budget_gib,
                                          loads)
        result["served_latency_ms"] = {"p50": result["serving"][f"load_{loads[0]}"]["latency_ms"]["p50"],
                                       "p99": result["serving"][f"load_{loads[0]}"]["latency_ms"]["p99"],
                                       "load": loads[0]} if loads else None

    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample ...")
        result["cpu_baseline"] = cpu_baseline(data0, st1.nli, full=args.cpu_full)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
