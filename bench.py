#!/usr/bin/env python3
"""Throughput of the PML-transmission double-sweep Helmholtz solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload layers] ...

One step = factor every padded strip (helm_factor) + solve all right-hand sides to a
1e-6 relative residual (helm_solve): the whole hot path on the inputs already resident
in HBM.  Metric: right-hand sides x interior grid points per second.  Prints one JSON
line.  Kernel durations come from HIP events recorded around every launch on the
solver's stream during the timed steps (helm_set_kernel_timing).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RHS·gridpts/s to 1e-6 residual, 2000² 2-D, c64-mixed vs c128 on 1 GPU"
PEAK = {"c64": 157.3, "c128": 78.6}          # dense MFMA TFLOP/s, FP32 / FP64
PHASES = ("phase_a", "phase_b", "phase_c", "factor_chunks", "factor_separators")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="layers", choices=["homogeneous_100", "lens_1000", "layers"])
    p.add_argument("--n", type=int, default=None, help="grid size for the layers family")
    p.add_argument("--nrhs", type=int, default=None)
    p.add_argument("--prec", default="mixed", choices=["mixed", "c128"])
    p.add_argument("--mode", default="reduced", choices=["reduced", "full"])
    p.add_argument("--chunk", type=int, default=0)
    p.add_argument("--tol", type=float, default=1e-6)
    p.add_argument("--no-cpu-baseline", action="store_true")
    return p.parse_args()


def workload(args):
    import workloads as W
    if args.workload == "homogeneous_100":
        wl = W.homogeneous_100()
    elif args.workload == "lens_1000":
        wl = W.lens_1000(nsrc=args.nrhs or 16)
    else:
        wl = W.layers(n=args.n or 2000, nsrc=args.nrhs or 64)
    return wl


def phase_flops(H, wl, nrhs):
    """Algorithmic real flops of one launch of each strip-solve phase and of the factor,
    averaged over strips (8 real flops per complex multiply-add)."""
    Ny = H.N_y
    m = H.chunk_rows
    P = -(-Ny // m)
    n_int = Ny - (P - 1)                    # interior rows over all chunks
    W2 = sum(w * w for w in H.strip_width) / len(H.strip_width)
    W3 = sum(w ** 3 for w in H.strip_width)
    fl = {
        # forward + backward block substitution: one W x W matvec per interior row each way
        "phase_a": 8.0 * W2 * nrhs * (2 * n_int - P),
        # separators: forward 2 matvecs (the first 1), backward 1 (the last none)
        "phase_b": 8.0 * W2 * nrhs * (2 * (P - 1) - 1 + (P - 2)) if P > 1 else 0.0,
        # spike corrections X~ x_above + Y~ x_below on every interior row that has them
        "phase_c": 8.0 * W2 * nrhs * (2 * n_int - (m - 1) - (Ny - (P - 1) * m)) if P > 1 else 0.0,
        # inverse (Gauss-Jordan, W^3) + top spike (2 W^3) + bottom spike (W^3) per interior row
        "factor_chunks": 8.0 * (W3 / len(H.strip_width)) * len(H.strip_width) * n_int * 4.0,
        "factor_separators": 8.0 * W3 * (P - 1) * 3.0,
    }
    return fl


def cpu_baseline(wl, iters_mean, budget_s=10.0):
    """The FP64 oracle on a bounded sample of the same workload, scaled to the job.

    Sample: assemble the global operator, factor padded strips with SuperLU (two solves
    each) for about `budget_s` seconds, and time 2 global residual evaluations.  One application of Algorithm 3
    is 2(J-1) strip solves plus 2 residual evaluations; the job is J strip factorisations
    plus, per right-hand side, (mean GPU iterations + 2) applications (the +2 standing for
    Algorithms 2 and 4)."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from oracle.assemble import assemble_global, assemble_strip
    from oracle.grid import geometry_from_workload

    t0 = time.time()
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    k2 = g.k2()
    rng = np.random.default_rng(0)
    t_fac, t_ss = [], []
    # strips in a fixed order until the sample has run about `budget_s` seconds (at least 2)
    order = [(k * 7919) % g.J for k in range(g.J)]
    for s in order:
        st = g.strips[s]
        ta = time.time()
        lu = spla.splu(assemble_strip(g, st, k2).tocsc(), permc_spec="COLAMD")
        t_fac.append(time.time() - ta)
        for _ in range(2):
            r = rng.standard_normal(g.N_y * st.W) + 0j
            ta = time.time()
            lu.solve(r)
            t_ss.append(time.time() - ta)
        if len(t_fac) >= 2 and time.time() - t0 > budget_s:
            break
    u = rng.standard_normal(g.N_y * g.N_x) + 0j
    ta = time.time()
    for _ in range(2):
        _ = u - A @ u
    t_res = (time.time() - ta) / 2
    t_fac_s = float(np.mean(t_fac))
    t_ss_s = float(np.mean(t_ss))
    t_ap = 2 * (g.J - 1) * t_ss_s + 2 * t_res
    est = t_fac_s * g.J + wl.nrhs * (iters_mean + 2.0) * t_ap
    return {
        "value": wl.nrhs * wl.n_x * wl.n_y / est, "unit": "RHS*gridpts/s", "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle (scipy SuperLU, single thread) pieces on {wl.name}: {len(t_fac)} of {g.J} strip "
                   f"factorisations ({t_fac_s:.2f} s each), {len(t_ss)} strip solves ({t_ss_s * 1e3:.1f} ms each), "
                   f"2 global residuals ({t_res * 1e3:.0f} ms each); scaled to J factorisations + "
                   f"nrhs x (mean GPU iterations {iters_mean:.1f} + 2) x [2(J-1) solves + 2 residuals]"),
        "est_job_s": est,
        "sample_wall_s": time.time() - t0,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1208_3956_amd import Helmholtz

    wl = workload(args)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    f = torch.from_numpy(wl.rhs()).to(dev)
    nrhs = f.shape[0]
    print(f"# {wl.name}: padded {wl.N_x}x{wl.N_y}, J={wl.J}, nrhs={nrhs}, {args.prec}/{args.mode}",
          file=sys.stderr, flush=True)
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                  prec=args.prec, mode=args.mode, chunk=args.chunk, device=dev)
    res = None
    for k in range(args.warmup):
        H.factor()
        res = H.solve(f, args.tol)
        print(f"# warmup {k}: iters {sorted(set(res.iters))} relres {max(res.relres):.2e}",
              file=sys.stderr, flush=True)
    H.set_kernel_timing(True)
    torch.cuda.synchronize()
    t_fac = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        ta = time.perf_counter()
        H.factor()
        torch.cuda.synchronize()
        t_fac += time.perf_counter() - ta
        res = H.solve(f, args.tol)
        print(f"# step {k}: iters {sorted(set(res.iters))} relres {max(res.relres):.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = H.kernel_times()
    H.set_kernel_timing(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    pts = nrhs * wl.n_x * wl.n_y
    value = pts / (ms_step / 1e3)
    solve_ms = ms_step - t_fac * 1e3 / args.steps
    dtype = "c64" if args.prec == "mixed" else "c128"

    # roofline of the costliest hot kernel class
    fl = phase_flops(H, wl, nrhs)
    dom = max(PHASES, key=lambda k: kt[k][1])
    cnt, ms = kt[dom]
    avg_s = ms / 1e3 / max(cnt, 1)
    ach = fl[dom] / avg_s / 1e12 if avg_s > 0 else 0.0
    peak = PEAK[dtype if dom.startswith("phase") else "c128"]
    roof = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": ach / peak, "traffic": None, "launches": cnt, "avg_launch_us": avg_s * 1e6,
            "flops_per_launch": fl[dom]}
    out = {
        "metric": METRIC, "value": value, "unit": "RHS*gridpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n_x, "nrhs": nrhs, "J": wl.J,
                   "pml_outer": wl.w_out, "pml_iface": wl.w, "prec": args.prec,
                   "mode": args.mode, "chunk_rows": H.chunk_rows, "tol": args.tol,
                   "step": "helm_factor + helm_solve"},
        "solve_only_value": pts / (solve_ms / 1e3), "solve_ms": solve_ms,
        "factor_ms": t_fac * 1e3 / args.steps,
        "iters": {"min": min(res.iters), "max": max(res.iters),
                  "mean": float(np.mean(res.iters))},
        "relres_max": max(res.relres), "restarts": res.restarts,
        "kernel_ms_per_step": {k: v[1] / args.steps for k, v in kt.items()},
        "roofline": roof,
    }
    H.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, float(np.mean(res.iters)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
