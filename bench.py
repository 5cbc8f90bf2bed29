"""Benchmark: SG apply GB/s and time to a 1e-8 residual, mixed vs double FGMRES, at P = 210.

Workload (synthetic, seeded): -div(a grad u) = 1 on the unit square, Q1 on a
513 x 513 grid (N = 261121 interior nodes), m = 6 KL terms of the separable
exponential covariance (L = 0.5), total degree p = 4 (P = 210, 54.8M
unknowns), sigma = 0.4, xi ~ U[-1, 1].

One step = one pass of the whole hot path on that system:
  * a burst of operator applies Y = A U in double (timed with HIP events on
    the library's stream; this is the reported SG apply GB/s), and
  * one block-triangular-preconditioned FGMRES(30) solve to a 1e-8 true
    relative residual with float V(2,2) cycles and double Krylov / residuals
    (the mixed-precision solve; its wall time is the time to 1e-8).
After the timed steps the all-double solve of the same problem is timed the
same way, for the mixed-vs-double comparison.  The oracle (CPU, double) is
timed on a bounded sample: its SG apply on the 65 x 65 copy of the workload
(same m, p, sigma; 833,490 unknowns).

Prints ONE JSON line.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SG apply GB/s + time to 1e-8 residual, mixed vs FP64 GMRES, at P=210"
HBM_PEAK_GBS = 8000.0


def apply_flops(N, P, m):
    """FP64 flops per double apply as the kernel computes it (FMA = 2): per node and mode the
    four cell residuals r_e (1 + 4 x 4), the m+1 stencil sums (4 FMAs each) and the 2m
    coupling gathers (one FMA each)."""
    return N * P * (17 + 8 * (m + 1) + 4 * m)


def apply_bytes(N, P, n, m, in_bytes=8, out_bytes=8):
    """Algorithmic bytes of one apply: read U, write Y, read the (m+1) cell coefficient fields once."""
    return N * P * (in_bytes + out_bytes) + 8 * n * n * (m + 1)


def traffic_from_profile(kernel_src, config):
    """HBM bytes per apply launch from committed rocprofv3 counter runs, if the kernel is unchanged."""
    path = os.path.join(ROOT, "profiles", f"apply_{config}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("config") != config:
        return None
    digest = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if rec.get("kernel_sha256") != digest:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(seconds=10.0):
    """Oracle SG apply (scipy CSR, double) on the 65 x 65 copy of the workload."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import sg_inputs
    from oracle import system
    c = sg_inputs.CONFIGS["c3_65"]
    o = system.build_problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"])
    A = system.assemble_A(o)
    x = sg_inputs.uniform_block(o.N, o.P, seed=1234).T.ravel().copy()
    y = A @ x
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        y = A @ x
        k += 1
    dt = (time.perf_counter() - t0) / k
    del y
    nbytes = apply_bytes(o.N, o.P, o.n, o.m)
    blas = sum(i.get("num_threads", 0) for i in threadpool_info()) or None
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} oracle applies (scipy CSR A @ x, {A.nnz} nnz) on the 65x65 copy of the workload "
                      f"(n=64, m=6, p=4, P=210, 833490 unknowns), {dt * 1e3:.1f} ms each; algorithmic bytes "
                      f"{nbytes / 1e6:.1f} MB per apply as for the GPU line",
            "host_cpu_count": os.cpu_count(), "blas_threads": blas}


def paper_table3(sgbt, stream):
    """Iterations and time to 1e-10 of the five solvers of Table 3 on the paper's own problem
    (P1 triangles, h = 1/64, m = 6, p = 4, L = 1, 833,490 unknowns) for sigma = 0.1 .. 0.4, with
    the four-colour and with the paper's lexicographic V(2,2), beside the printed counts."""
    golden = {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_numbers.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if "=" in line:
                k, v = line.split("=", 1)
                golden[k.strip()] = v.strip()
    solvers = [("block GS", dict(solver="bgs", precond="tri")), ("BD-PCG", dict(solver="pcg", precond="diag")),
               ("BT-GPCG", dict(solver="gpcg", precond="tri")),
               ("BT-GMRes(10)", dict(solver="fgmres", precond="tri", restart=10)),
               ("BS-PCG", dict(solver="pcg", precond="sym"))]
    rows = {}
    for sigma in (0.1, 0.2, 0.3, 0.4):
        row = {"paper_iters": [int(v) for v in golden[f"table3_iters_sigma_{sigma}"].split()]}
        for colour, tag in (("four", ""), ("lex", "_lex")):
            pr = sgbt.Problem(64, 6, 4, sigma, corr_len=1.0, coarsest=4, disc="p1", colour=colour, stream=stream)
            F = pr.rhs()
            X = pr.empty()
            its, ms = [], []
            for _, kw in solvers:
                pr.solve(F, X, rtol=1e-10, max_it=300, **kw)  # warm
                _, info = pr.solve(F, X, rtol=1e-10, max_it=300, **kw)
                its.append(info["iters"] if info["status"] == 0 else None)
                ms.append(info["t_total_ms"])
            pr.close()
            row["iters" + tag] = its
            row["ms" + tag] = ms
        rows[str(sigma)] = row
    return {"solvers": [name for name, _ in solvers], "rtol": 1e-10, "unknowns": 833490,
            "smoothers": {"iters": "four-colour V(2,2)", "iters_lex": "lexicographic V(2,2), as in Sec. 6"},
            "sigma": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--burst", type=int, default=12, help="double applies timed per step")
    ap.add_argument("--mode", default="full", choices=["full", "apply", "paper"],
                    help="apply: only the double apply loop (for profiler counter runs); "
                         "paper: only the Sec. 6 Table 3 solvers")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-paper", action="store_true", help="skip the Sec. 6 iteration-count table")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(each box has one MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1304_1755_amd as sgbt
    import sg_inputs

    torch.cuda.set_device(0)
    c = sg_inputs.CONFIGS[args.config]
    stream = torch.cuda.current_stream()
    if args.mode == "paper":
        print(json.dumps({"mode": "paper", "paper_sec6_table3": paper_table3(sgbt, stream)}))
        return
    prob = sgbt.Problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"], colour="four", nu1=2, nu2=2,
                        coarsest=8, stream=stream)
    N, P, n, m = prob.N, prob.P, c["n"], c["m"]
    # inputs resident in HBM before the timed region (seeded device generator)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    U = torch.rand((N, P), dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
    Y = torch.empty_like(U)
    F = prob.rhs()
    X = torch.empty_like(U)
    nbytes = apply_bytes(N, P, n, m)

    if args.mode == "apply":
        a = torch.empty(N * P, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.warmup):
            prob.apply(U, Y)
        torch.cuda.synchronize()
        b.copy_(a)  # plain copy of known size (2 * 8 * N * P bytes) for counter calibration
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            prob.apply(U, Y)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"mode": "apply", "ms_per_apply_wall": dt * 1e3, "bytes": nbytes,
                          "copy_bytes": 16 * N * P}))
        return

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.burst)]

    def step(timed):
        for s, e in ev:
            s.record(stream)
            prob.apply(U, Y)
            e.record(stream)
        _, info = prob.solve(F, X, precond="tri", prec=sgbt.SG_MIXED, restart=c["restart"], rtol=1e-8,
                             max_it=300)
        if timed:
            torch.cuda.synchronize()
            return [s.elapsed_time(e) for s, e in ev], info
        return None, info

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    progress(f"setup done: N={N} P={P}; warmup {args.warmup}")
    for _ in range(args.warmup):
        _, winfo = step(False)
        progress(f"warmup solve: {winfo['iters']} it, residual {winfo['rel_res_true']:.2e}, "
                 f"{winfo['t_total_ms']:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    apply_ms, solves = [], []
    for _ in range(args.steps):
        ms, info = step(True)
        apply_ms += ms
        solves.append(info)
        progress(f"step: apply {np.mean(ms):.3f} ms, mixed solve {info['iters']} it {info['t_total_ms']:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3

    # all-double solve of the same problem, same algorithm (outside the timed steps)
    d_solves = []
    for _ in range(max(1, args.steps)):
        _, info = prob.solve(F, X, precond="tri", prec=sgbt.SG_F64, restart=c["restart"], rtol=1e-8, max_it=300)
        d_solves.append(info)
        progress(f"double solve: {info['iters']} it {info['t_total_ms']:.1f} ms")
    torch.cuda.synchronize()

    avg_apply_ms = float(np.mean(apply_ms))
    med_apply_ms = float(np.median(apply_ms))
    achieved = nbytes / (avg_apply_ms * 1e-3) / 1e9
    t_mixed = float(np.median([s["t_total_ms"] for s in solves])) / 1e3
    t_f64 = float(np.median([s["t_total_ms"] for s in d_solves])) / 1e3
    traffic = traffic_from_profile(os.path.join(ROOT, "paper_1304_1755_amd", "csrc", "sg_apply_kernel.h"), args.config)
    out = {
        "metric": METRIC,
        "value": achieved,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: Q1 {n + 1}x{n + 1} grid (N={N}), m={m}, p={c['p']}, P={P} "
                               f"({N * P} unknowns), sigma={c['sigma']}, L={c['corr_len']}; step = {args.burst} "
                               f"double SG applies + one mixed B_T-FGMRES({c['restart']}) V(2,2) solve to 1e-8",
                   "N": N, "P": P, "unknowns": N * P},
        "time_to_1e-8_s": {"mixed": t_mixed, "fp64": t_f64, "speedup_mixed_vs_fp64": t_f64 / t_mixed,
                           "iters_mixed": solves[-1]["iters"], "iters_fp64": d_solves[-1]["iters"],
                           "true_rel_res_mixed": solves[-1]["rel_res_true"],
                           "true_rel_res_fp64": d_solves[-1]["rel_res_true"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sg_apply (double in/out)", "algorithmic_bytes_per_launch": nbytes,
                     "avg_launch_ms": avg_apply_ms, "median_launch_ms": med_apply_ms,
                     "launches_timed": len(apply_ms),
                     "fp64_tflops": apply_flops(N, P, m) / (avg_apply_ms * 1e-3) / 1e12,
                     "fp64_vector_peak_tflops": 78.6},
    }
    prob.close()
    if not args.no_paper:
        progress("the paper's Sec. 6 problem (P1, h = 1/64, m = 6, p = 4): Table 3 solvers")
        out["paper_sec6_table3"] = paper_table3(sgbt, stream)
    if not args.no_cpu:
        progress("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
