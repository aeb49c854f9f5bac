#!/usr/bin/env python3
"""Throughput of the PML-transmission double-sweep Helmholtz solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload layers] ...

One step = factor every padded strip (helm_factor) + solve all right-hand sides to a
1e-6 relative residual (helm_solve): the whole hot path on the inputs already resident
in HBM.  Metric: right-hand sides x interior grid points per second.  Prints one JSON
line.  One untimed step with HIP events around every hot-kernel launch gives the per-class
breakdown and names the dominant kernel class; during the timed steps only that class is
bracketed with events on the solver's stream (helm_set_kernel_timing), so its average
launch duration is measured live over the timed region while the rest runs undisturbed.
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
    p.add_argument("--workload", default="layers",
                   choices=["homogeneous_100", "lens_1000", "layers", "layers_uneven_batch", "smooth_3d"])
    p.add_argument("--n", type=int, default=None, help="grid size for the layers family")
    p.add_argument("--nrhs", type=int, default=None)
    p.add_argument("--prec", default="mixed", choices=["mixed", "c128"])
    p.add_argument("--mode", default="reduced", choices=["reduced", "full"])
    p.add_argument("--chunk", type=int, default=0,
                   help="rows per chunk of the strip solver; 0 = autotuned before the timed steps")
    p.add_argument("--tune-candidates", default="16,24,32,40,48",
                   help="chunk sizes the autotuner times (2-D)")
    p.add_argument("--tol", type=float, default=1e-6)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-c128-leg", action="store_true",
                   help="skip the complex128 comparison legs (batched and one RHS per solve)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a plain device-to-device copy of MIB MiB three times and exit "
                        "(reference dispatch for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return p.parse_args()


def workload(args):
    import workloads as W
    if args.workload == "homogeneous_100":
        wl = W.homogeneous_100()
    elif args.workload == "lens_1000":
        wl = W.lens_1000(nsrc=args.nrhs or 16)
    elif args.workload == "smooth_3d":
        wl = W.smooth_3d(n=args.n or 80, nsrc=args.nrhs or 32)
    else:
        wl = W.layers(n=args.n or 2000, nsrc=args.nrhs or 64)
    return wl


def phase_flops(H, wl, nrhs):
    """Algorithmic real flops of one launch of each strip-solve phase and of the factor,
    averaged over strips (8 real flops per complex multiply-add).  In 3-D one timed
    phase-A launch is a whole slab solve (2 N_y - 1 plane products with the B x B inverses,
    B = W N_z) and one timed factor unit is the whole factorisation (B^3 multiply-adds of
    Gauss-Jordan per slab and plane)."""
    Ny = H.N_y
    slot = H.strip_factor_slot               # identical strips share one factorisation
    reps = [slot.index(u) for u in range(max(slot) + 1)]
    if H.dim == 3:
        B = [w * H.N_z for w in H.strip_width]
        B2 = sum(b * b for b in B) / len(B)
        return {"phase_a": 8.0 * B2 * nrhs * (2 * Ny - 1), "phase_b": 0.0, "phase_c": 0.0,
                "factor_chunks": 8.0 * sum(B[r] ** 3 for r in reps) * Ny, "factor_separators": 0.0}
    m = H.chunk_rows
    P = -(-Ny // m)
    n_int = Ny - (P - 1)                    # interior rows over all chunks
    W2 = sum(w * w for w in H.strip_width) / len(H.strip_width)
    W3 = sum(H.strip_width[r] ** 3 for r in reps)
    fl = {
        # forward + backward block substitution: one W x W matvec per interior row each way
        "phase_a": 8.0 * W2 * nrhs * (2 * n_int - P),
        # separators: forward 2 matvecs (the first 1), backward 1 (the last none)
        "phase_b": 8.0 * W2 * nrhs * (2 * (P - 1) - 1 + (P - 2)) if P > 1 else 0.0,
        # spike corrections X~ x_above + Y~ x_below on every interior row that has them
        "phase_c": 8.0 * W2 * nrhs * (2 * n_int - (m - 1) - (Ny - (P - 1) * m)) if P > 1 else 0.0,
        # inverse (Gauss-Jordan, W^3) + top spike (2 W^3) + bottom spike (W^3) per interior row
        "factor_chunks": 8.0 * W3 * n_int * 4.0,
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
            r = rng.standard_normal(int(np.prod(g.strip_shape(st)))) + 0j
            ta = time.time()
            lu.solve(r)
            t_ss.append(time.time() - ta)
        if len(t_fac) >= 2 and time.time() - t0 > budget_s:
            break
    u = rng.standard_normal(int(np.prod(g.field_shape))) + 0j
    ta = time.time()
    for _ in range(2):
        _ = u - A @ u
    t_res = (time.time() - ta) / 2
    t_fac_s = float(np.mean(t_fac))
    t_ss_s = float(np.mean(t_ss))
    t_ap = 2 * (g.J - 1) * t_ss_s + 2 * t_res
    est = t_fac_s * g.J + wl.nrhs * (iters_mean + 2.0) * t_ap
    return {
        "value": wl.nrhs * wl.n_points / est, "unit": "RHS*gridpts/s", "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle (scipy SuperLU, single thread) pieces on {wl.name}: {len(t_fac)} of {g.J} strip "
                   f"factorisations ({t_fac_s:.2f} s each), {len(t_ss)} strip solves ({t_ss_s * 1e3:.1f} ms each), "
                   f"2 global residuals ({t_res * 1e3:.0f} ms each); scaled to J factorisations + "
                   f"nrhs x (mean GPU iterations {iters_mean:.1f} + 2) x [2(J-1) solves + 2 residuals]"),
        "est_job_s": est,
        "sample_wall_s": time.time() - t0,
    }


KERNEL_SOURCES = ("paper_1208_3956_amd/csrc/kernels_solve.hip",
                  "paper_1208_3956_amd/csrc/kernels_vec.hip",
                  "paper_1208_3956_amd/csrc/helm_internal.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(cls, wl, nrhs, prec, prefix=""):
    """HBM bytes per launch of kernel class `cls` from the committed counter summary of this
    workload, or None when there is none or the kernel sources changed since it was taken.
    The summary holds FETCH_SIZE and WRITE_SIZE per dispatch already scaled by the copy
    calibration, and the sha256 of the kernel sources it was measured on; `prefix` selects
    another kernel's entries in the same summary (the stencil's: "stencil_")."""
    import re
    path = os.path.join(ROOT, "profiles", f"{cls}_hbm_traffic_{wl.name}_nrhs{nrhs}_{prec}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    want = {}
    for key in ("source_sha256", f"{prefix}fetch_bytes_per_launch", f"{prefix}write_bytes_per_launch"):
        m = re.search(rf"^{key}:\s*(\S+)\s*$", text, re.M)
        if not m:
            return None
        want[key] = m.group(1)
    if want["source_sha256"] != kernel_source_hash():
        return None
    return float(want[f"{prefix}fetch_bytes_per_launch"]) + float(want[f"{prefix}write_bytes_per_launch"])


def algorithmic_bytes(H, nrhs, prec):
    """HBM bytes that one phase-A launch must move at least: the factor blocks G_l of every
    interior row read once per direction, the right-hand side read once, the chunk result
    written once (complex64: 8 B, complex128: 16 B per value)."""
    b = 8 if prec == "mixed" else 16
    Ny, m = H.N_y, H.chunk_rows
    P = -(-Ny // m)
    n_int = Ny - (P - 1)
    W = sum(H.strip_width) / len(H.strip_width)
    return b * (2.0 * W * W * n_int + 2.0 * W * Ny * nrhs)


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                      "dispatches": 3}), flush=True)


def stencil_roofline(H, wl, f, reps=5):
    """HBM roofline of the full-field stencil r = f - A u (helm_apply_A) on the bench's
    right-hand sides: algorithmic bytes = read u, read f, write r (16 B each per point and
    right-hand side) + k^2 once (8 B per point), over its average launch (HIP events)."""
    import torch
    H.set_kernel_timing(True, classes=["stencil"])
    for _ in range(reps):
        out = H.apply_A(f, f)
    torch.cuda.synchronize()
    cnt, ms = H.kernel_times()["stencil"]
    H.set_kernel_timing(False)
    del out
    avg_s = ms / 1e3 / max(cnt, 1)
    pts = wl.N_x * wl.N_y * wl.N_z if wl.dim == 3 else wl.N_x * wl.N_y
    nbytes = f.shape[0] * pts * 48 + pts * 8
    ach = nbytes / avg_s / 1e9
    return {"kernel": "k_apply_A", "bound": "hbm", "achieved": ach, "peak": 8000.0, "unit": "GB/s",
            "frac": ach / 8000.0, "avg_launch_us": avg_s * 1e6, "bytes_per_launch": nbytes,
            "launches": cnt}


def c128_legs(wl, f, tol, plain_rhs=2):
    """Complex128 comparison on the same workload: the batched solve (all right-hand sides in
    one helm_solve) and the plain path (one right-hand side per helm_solve), each after a
    factorisation, one timed pass; the plain path is timed on `plain_rhs` right-hand sides and
    scaled per right-hand side (the metric is additive over independent right-hand sides)."""
    import numpy as np
    import torch
    from paper_1208_3956_amd import Helmholtz
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                  prec="c128", mode="reduced", device="cuda:0")
    if wl.dim == 2:
        H.autotune(f, reps=1, cache=None)     # factors with its own best chunk size
    else:
        H.factor()
    torch.cuda.synchronize()
    pts_rhs = wl.n_points
    ta = time.perf_counter()
    res = H.solve(f, tol)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - ta
    t_plain = 0.0
    it_plain = []
    for k in range(plain_rhs):
        ta = time.perf_counter()
        r1 = H.solve(f[k:k + 1], tol)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - ta
        it_plain.append(r1.iters[0])
    H.close()
    print(f"# c128: batched {t_batch * 1e3:.0f} ms, plain {t_plain / plain_rhs * 1e3:.0f} ms per RHS",
          file=sys.stderr, flush=True)
    return {
        "batched": {"solve_only_value": f.shape[0] * pts_rhs / t_batch, "solve_ms": t_batch * 1e3,
                    "iters_mean": float(np.mean(res.iters)), "relres_max": max(res.relres)},
        "plain_one_rhs_per_solve": {"solve_only_value": pts_rhs * plain_rhs / t_plain,
                                    "ms_per_rhs": t_plain / plain_rhs * 1e3,
                                    "rhs_timed": plain_rhs, "iters": it_plain},
    }


def batch_main(args):
    """Eight uneven layered problems (500^2 ... 2000^2, 8 RHS each): one step = factor all +
    solve all concurrently (helm_solve_batch, one stream per problem); the same handles are
    also solved one after another for comparison."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1208_3956_amd import Helmholtz, solve_batch
    wls = W.layers_uneven_batch()
    dev = "cuda:0"
    torch.cuda.set_device(0)
    fs = [torch.from_numpy(wl.rhs()).to(dev) for wl in wls]
    streams = [torch.cuda.Stream(dev) for _ in wls]
    Hs = [Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                    prec=args.prec, mode=args.mode, chunk=args.chunk, device=dev, stream=s)
          for wl, s in zip(wls, streams)]
    pts = sum(f.shape[0] * wl.n_x * wl.n_y for wl, f in zip(wls, fs))

    def step(concurrent):
        for H in Hs:
            H.factor()
        for H in Hs:
            H.stream.synchronize()
        if concurrent:
            return solve_batch(Hs, fs, args.tol)
        return [H.solve(f, args.tol) for H, f in zip(Hs, fs)]

    for k in range(args.warmup):
        print(f"# batch warmup {k}: concurrent", file=sys.stderr, flush=True)
        step(True)
        print(f"# batch warmup {k}: sequential", file=sys.stderr, flush=True)
        step(False)
    torch.cuda.synchronize()
    print("# batch timed: concurrent", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step(True)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / args.steps
    print("# batch timed: sequential", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res_s = step(False)
    torch.cuda.synchronize()
    t_s = (time.perf_counter() - t0) / args.steps
    for H in Hs:
        H.close()
    out = {
        "metric": "RHS*gridpts/s to 1e-6 residual, uneven batch of 8 layered 2-D problems (500^2..2000^2, 8 RHS each)",
        "value": pts / t_b, "unit": "RHS*gridpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_b * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64" if args.prec == "mixed" else "c128", "data": "synthetic",
        "config": {"workload": "layers_uneven_batch", "sizes": [wl.n_x for wl in wls],
                   "J": [wl.J for wl in wls], "nrhs_each": 8, "prec": args.prec, "mode": args.mode,
                   "step": "helm_factor (each) + helm_solve_batch"},
        "sequential_value": pts / t_s, "sequential_ms_per_step": t_s * 1e3,
        "iters": [float(np.mean(r.iters)) for r in res],
        "relres_max": max(max(r.relres) for r in res + res_s),
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload == "layers_uneven_batch":
        batch_main(args)
        return
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
    tuned = None
    if args.chunk == 0 and wl.dim == 2:
        # outside the timed region: one GMRES iteration's operator timed per candidate
        cand = [int(x) for x in args.tune_candidates.split(",") if x.strip()]
        tuned = H.autotune(f, candidates=cand, reps=2, cache=None)
        print(f"# autotune: chunk {tuned['chunk_rows']} "
              f"({', '.join(f'{c}: {t:.1f} ms' for c, t in tuned['ms_per_apply'].items())})",
              file=sys.stderr, flush=True)
    res = None
    for k in range(args.warmup):
        H.factor()
        res = H.solve(f, args.tol)
        print(f"# warmup {k}: iters {sorted(set(res.iters))} relres {max(res.relres):.2e}",
              file=sys.stderr, flush=True)
    # breakdown step: every hot-kernel class timed, names the dominant one
    H.set_kernel_timing(True)
    H.factor()
    H.solve(f, args.tol)
    torch.cuda.synchronize()
    kt_all = H.kernel_times()
    dom = max(PHASES, key=lambda k: kt_all[k][1])
    H.set_kernel_timing(True, classes=[dom])
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
    pts = nrhs * wl.n_points
    value = pts / (ms_step / 1e3)
    solve_ms = ms_step - t_fac * 1e3 / args.steps
    dtype = "c64" if args.prec == "mixed" else "c128"

    # roofline of the costliest hot kernel class
    fl = phase_flops(H, wl, nrhs)
    cnt, ms = kt[dom]
    avg_s = ms / 1e3 / max(cnt, 1)
    ach = fl[dom] / avg_s / 1e12 if avg_s > 0 else 0.0
    # the strip solves run in the working precision; the 2-D factor computes in FP64; the
    # 3-D mixed factor in FP32 unless it fell back to the FP64 route
    if dom.startswith("phase"):
        arith = dtype
    else:
        arith = "c64" if (wl.dim == 3 and args.prec == "mixed" and H.factor_path == 1) else "c128"
    peak = PEAK[arith]
    roof = {"kernel": dom, "bound": "mfma", "arith": "fp32" if arith == "c64" else "fp64",
            "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": ach / peak, "traffic": profiled_traffic(dom, wl, nrhs, args.prec),
            "launches": cnt, "avg_launch_us": avg_s * 1e6, "flops_per_launch": fl[dom]}
    if dom == "phase_a":
        roof["algorithmic_bytes_per_launch"] = algorithmic_bytes(H, nrhs, args.prec)
    # the factorisation's MFMA use, from the breakdown step (whatever class dominates)
    fcnt, fms = kt_all["factor_chunks"]
    farith = "c64" if (wl.dim == 3 and args.prec == "mixed" and H.factor_path == 1) else "c128"
    fach = fl["factor_chunks"] * fcnt / (fms / 1e3) / 1e12 if fms > 0 else 0.0
    factor_roof = {"kernel": "factor_chunks", "arith": "fp32" if farith == "c64" else "fp64",
                   "achieved": fach, "peak": PEAK[farith], "unit": "TFLOP/s",
                   "frac": fach / PEAK[farith], "launches": fcnt, "ms": fms,
                   "flops_per_launch": fl["factor_chunks"],
                   "from": "one untimed step with every class timed"}
    metric = METRIC if wl.dim == 2 else "RHS*gridpts/s to 1e-6 residual, 80^3 3-D, c64-mixed, 1 GPU"
    out = {
        "metric": metric, "value": value, "unit": "RHS*gridpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n_x, "dim": wl.dim, "nrhs": nrhs, "J": wl.J,
                   "pml_outer": wl.w_out, "pml_iface": wl.w, "prec": args.prec,
                   "mode": args.mode, "chunk_rows": H.chunk_rows, "tol": args.tol,
                   "autotune": tuned, "factor_path": H.factor_path if wl.dim == 3 else None,
                   "factor_slots": H.factor_slots,
                   "step": "helm_factor + helm_solve"},
        "solve_only_value": pts / (solve_ms / 1e3), "solve_ms": solve_ms,
        "factor_ms": t_fac * 1e3 / args.steps,
        "iters": {"min": min(res.iters), "max": max(res.iters),
                  "mean": float(np.mean(res.iters))},
        "relres_max": max(res.relres), "restarts": res.restarts,
        "kernel_ms_per_step": {k: v[1] for k, v in kt_all.items()},
        "kernel_ms_per_step_from": "one untimed step with every class timed",
        "roofline": roof,
        "factor_roofline": factor_roof,
        "stencil_roofline": dict(stencil_roofline(H, wl, f),
                                 traffic=profiled_traffic("phase_a", wl, nrhs, args.prec, "stencil_")),
    }
    H.close()
    if args.prec == "mixed" and not args.no_c128_leg:
        out["c128"] = c128_legs(wl, f, args.tol)
        out["mixed_vs_c128_batched"] = out["solve_only_value"] / out["c128"]["batched"]["solve_only_value"]
        out["mixed_vs_c128_plain"] = (out["solve_only_value"]
                                      / out["c128"]["plain_one_rhs_per_solve"]["solve_only_value"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, float(np.mean(res.iters)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
