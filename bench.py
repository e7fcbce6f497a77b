#!/usr/bin/env python
"""Benchmark of the interior point solver on one MI355X.

Workload: 2D Poisson on the 511 x 511 interior grid (261,121 nodes per field,
1,044,484 unknowns per Newton system) with the L1 term, control box
u in [-5, 5] and state box y in [-0.2, 0.3]; y_d is a sum of 8 seeded sine
modes; alpha = 1e-4, beta = 1e-3, sigma = 0.2 (workloads.poisson2d_511).

One step = one complete interior point solve (every Newton system, Krylov
iteration, preconditioner application and update of Algorithm A.1), inputs
already resident in HBM.  The headline path runs MINRES + P_D with FP32
V-cycles; the plain FP64 V-cycle variant is timed beside it.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the roofline kernel from rocprofv3 FETCH_SIZE/WRITE_SIZE
# runs (profiles/k_minres_k1_poisson2d_511_pmc.md), valid while the kernel
# sources hash to the value they were measured with.
TRAFFIC = {"kernel": 6, "N": 511, "bytes": 140424333.4, "source_sha": "4c06722113282728"}
KERNEL_NAMES = {0: "k_saddle (saddle matvec)", 1: "k_mg_jacobi (finest-level smoothing sweep)",
                2: "k_minres_k2 (Lanczos + diagonal preconditioner)", 3: "one V-cycle",
                4: "k_mg_down2d (finest level: smoothing + residual + restriction)",
                5: "k_mg_up2d (finest level: prolongation + smoothing)",
                6: "k_minres_k1 (MINRES update + saddle matvec + dots)"}


def measured_traffic(args):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1806_05896_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("kernels_krylov.hip", "common.h"))
    sha = hashlib.sha256(src).hexdigest()[:16]
    if args.kernel == TRAFFIC["kernel"] and args.N == TRAFFIC["N"] and sha == TRAFFIC["source_sha"]:
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


def cpu_baseline(data, nli):
    """The oracle (SuperLU Newton solve) on a bounded sample: the first IPM
    iteration of the same 511 x 511 problem, scaled to solves/s by the
    number of IPM iterations of a full solve."""
    import numpy as np  # noqa: F401
    import oracle
    from oracle.fd import discretize
    from oracle.ipm import IPMOptions, initial_state, ipm_step
    opts = IPMOptions(sigma=data.sigma)
    t0 = time.perf_counter()
    disc = discretize(data)
    st = initial_state(data, opts)
    st, _ = ipm_step(data, disc, st, opts, st.mu * opts.sigma)
    t = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS")
    return {"value": 1.0 / (t * nli), "unit": "IPM solves/s", "cores": 1,
            "kind": "oracle",
            "sample": f"1 of {nli} IPM iterations of the 511x511 workload (SuperLU on the eliminated SPD "
                      f"Newton system, {t:.1f} s), scaled by {nli}; SuperLU factorization is single-threaded"
                      + (f"; OMP_NUM_THREADS={threads}" if threads else "")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 V-cycle variant")
    ap.add_argument("--kernel", type=int, default=6, help="kernel id for the roofline figure")
    ap.add_argument("--N", type=int, default=511)
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
    data = W.poisson2d_511(seed=0, N=args.N)
    prob = Problem(data)
    opts = Options(sigma=data.sigma, mg_precision="fp32")
    if args.pmc_probe:
        # the roofline kernel at a mid-solve Newton state, then a plain copy of known size
        # (1 GiB, larger than the 256 MB Infinity Cache) that calibrates the byte counters
        for k in range(6):
            prob.ipm_step(opts.sigma ** (k + 1), opts)
        prob.newton_setup(opts.sigma ** 7, opts)
        ms, nbytes = prob.time_kernel(args.kernel, reps=20, opts=opts)
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": KERNEL_NAMES[args.kernel], "algorithmic_bytes": nbytes,
                          "copy_bytes_each_direction": src.numel() * 8}))
        prob.close()
        return
    log(f"workload poisson2d_511 N={data.N} n={data.n}")
    t, lat, its, st, rc = time_solves(prob, opts, args.steps, args.warmup, torch)
    u32 = prob.query("u")
    solves_per_s = args.steps / t
    result = {
        "metric": "IPM solves/s (2D Poisson 511^2, L1 + control and state boxes)",
        "value": solves_per_s,
        "unit": "IPM solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded sine-mode desired state, workloads.poisson2d_511)",
        "config": {"workload": f"poisson2d_511: 2D Poisson {data.N}x{data.N} interior, alpha=1e-4, beta=1e-3, "
                               "u in [-5,5], y in [-0.2,0.3], sigma=0.2, IPM tol 1e-6",
                   "krylov": "minres", "precond": "P_D", "mg_precision": "fp32", "vcycles": 1,
                   "nu_pre": 2, "nu_post": 2, "krylov_tol": 1e-10, "status": rc},
        "krylov_its_per_s": its / t,
        "nli": st.nli,
        "krylov_its_per_solve": its / args.steps,
        "krylov_its_per_ipm_step": st.hist_krylov[:st.nli],
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
    }

    # roofline of the dominant kernel, timed live with HIP events on the solve stream
    prob.newton_setup(st.mu if st.mu > 0 else 1e-6, opts)
    ms, nbytes = prob.time_kernel(args.kernel, reps=200, opts=opts, stream=torch.cuda.current_stream())
    achieved = nbytes / (ms * 1e-3) / 1e9
    result["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args),
                          "kernel": KERNEL_NAMES[args.kernel], "avg_us": ms * 1e3,
                          "algorithmic_bytes_per_launch": nbytes}
    kern = {}
    for k in (0, 2, 3, 4, 5, 6):
        ms_k, b_k = prob.time_kernel(k, reps=100, opts=opts, stream=torch.cuda.current_stream())
        kern[KERNEL_NAMES[k]] = {"avg_us": ms_k * 1e3, "GB/s": b_k / (ms_k * 1e-3) / 1e9}
    result["kernels"] = kern

    if not args.no_fp64:
        opts64 = Options(sigma=data.sigma, mg_precision="fp64")
        t64, lat64, its64, st64, rc64 = time_solves(prob, opts64, max(2, args.steps // 2), 1, torch)
        u64 = prob.query("u")
        n64 = max(2, args.steps // 2)
        result["fp64_vcycles"] = {"solves_per_s": n64 / t64, "krylov_its_per_solve": its64 / n64,
                                  "nli": st64.nli, "status": rc64,
                                  "rel_l2_u_vs_fp32_path": float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64))}

    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample ...")
        result["cpu_baseline"] = cpu_baseline(data, st.nli)
    prob.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
