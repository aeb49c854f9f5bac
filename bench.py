#!/usr/bin/env python3
"""Throughput of the PML-transmission double-sweep Helmholtz solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload layers] ...

One step = factor every padded strip (helm_factor) + solve all right-hand sides to a
1e-6 relative residual (helm_solve): the whole hot path on the inputs already resident
in HBM.  Metric: right-hand sides x interior grid points per second.  Prints one JSON
line.  The timed steps run the configured path untouched (in reduced mode each GMRES
iteration replays Algorithm 3 from a HIP graph).  Then one step with HIP events around
every hot-kernel launch gives the per-class breakdown and names the dominant kernel class,
and a few more steps bracket only that class with events on the solver's stream
(helm_set_kernel_timing) for its average launch duration.
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
    p.add_argument("--sweep", default="double", choices=["double", "concurrent"],
                   help="double: the paper's P; concurrent: P_c (both sweeps on f at once)")
    p.add_argument("--chunk", type=int, default=0,
                   help="rows per chunk of the strip solver; 0 = autotuned before the timed steps")
    p.add_argument("--tune-candidates", default="16,24,32,40,48",
                   help="chunk sizes the autotuner times (2-D)")
    p.add_argument("--tol", type=float, default=1e-6)
    p.add_argument("--roofline-steps", type=int, default=2,
                   help="steps run after the timed ones with the dominant kernel class event-timed")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-baseline", default="sample", choices=["sample", "full"],
                   help="sample: re-time a bounded oracle sample and scale the committed record of the "
                        "oracle's whole job; full: run the oracle's whole job now (minutes)")
    p.add_argument("--oracle-record-out", default=None,
                   help="with --cpu-baseline full: also write the job record (Markdown) here")
    p.add_argument("--no-lens-leg", action="store_true",
                   help="skip the 1000^2 Gaussian-lens leg (complex64-mixed and complex128)")
    p.add_argument("--no-3d-leg", action="store_true",
                   help="skip the 80^3 smooth-medium leg (complex64-mixed, reduced)")
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


def _oracle_solve_one(k):
    """Worker of the all-cores leg: the oracle's DD-GMRES on right-hand side k with the
    factorisations inherited from the parent (fork)."""
    from oracle.solve import solve_dd_reduced
    g, A, S, f = _ORACLE_CTX
    t = time.time()
    r = solve_dd_reduced(g, f[k], 1e-6, S=S, A=A)
    return k, time.time() - t, r.iters, r.relres


_ORACLE_CTX = None


def _strip_pieces(g, k2, strips, nsolve=2):
    """SuperLU factorisation of the given strips and nsolve solves each (seconds, means)."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from oracle.assemble import assemble_strip
    rng = np.random.default_rng(0)
    tf, ts = [], []
    for s in strips:
        st = g.strips[s]
        ta = time.time()
        lu = spla.splu(assemble_strip(g, st, k2).tocsc(), permc_spec="COLAMD")
        tf.append(time.time() - ta)
        for _ in range(nsolve):
            r = rng.standard_normal(int(np.prod(g.strip_shape(st)))) + 0j
            ta = time.time()
            lu.solve(r)
            ts.append(time.time() - ta)
    return float(np.mean(tf)), float(np.mean(ts))


SAMPLE_STRIPS = (0, 1, 2)


def oracle_job(wl, max_cores=16):
    """The FP64 oracle's whole job on the host, as it stands (scipy SuperLU, one thread per
    process): assemble the global operator, factor every padded strip (StripSolvers), then
    the reduced DD-GMRES of Algorithm 5 on right-hand side 0 end to end with its own
    iteration count (1 core); then C = min(cores, max_cores) processes forked after the
    factorisation each solve one further right-hand side (all cores).  Also times the
    bounded sample the default run re-times (SAMPLE_STRIPS factorisations and solves)."""
    global _ORACLE_CTX
    import multiprocessing as mp
    from oracle.assemble import assemble_global
    from oracle.dd import StripSolvers
    from oracle.grid import geometry_from_workload
    from oracle.solve import solve_dd_reduced

    t0 = time.time()
    g = geometry_from_workload(wl)
    A = assemble_global(g)
    t_asm = time.time() - t0
    t_sfac, t_ssol = _strip_pieces(g, g.k2(), SAMPLE_STRIPS)
    ta = time.time()

    def progress(done, J):
        if done % 8 == 0 or done == J:
            print(f"# oracle: {done}/{J} strips factored ({time.time() - ta:.0f} s)", file=sys.stderr, flush=True)
    S = StripSolvers(g, progress=progress)
    t_fac = time.time() - ta
    cores = max(1, min(max_cores, os.cpu_count() or 1))
    nsolve = min(wl.nrhs, cores + 1)
    f = wl.rhs(list(range(nsolve)))
    ta = time.time()
    r0 = solve_dd_reduced(g, f[0], 1e-6, S=S, A=A)
    t_one = time.time() - ta
    print(f"# oracle: assemble {t_asm:.1f} s, factor {g.J} strips {t_fac:.1f} s, one RHS {t_one:.1f} s "
          f"({r0.iters} iterations)", file=sys.stderr, flush=True)
    C = min(cores, nsolve - 1)
    t_par, it_par = None, []
    if C >= 2:
        _ORACLE_CTX = (g, A, S, f)
        old = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
        os.environ["OMP_NUM_THREADS"] = os.environ["OPENBLAS_NUM_THREADS"] = "1"
        try:
            ta = time.time()
            res = []
            with mp.get_context("fork").Pool(C) as pool:
                for r in pool.imap_unordered(_oracle_solve_one, range(1, C + 1)):
                    res.append(r)
                    print(f"# oracle: right-hand side {r[0]} done in {r[1]:.0f} s ({r[2]} iterations)",
                          file=sys.stderr, flush=True)
            t_par = time.time() - ta
            it_par = [r[2] for r in res]
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
            _ORACLE_CTX = None
        print(f"# oracle: {C} RHS on {C} processes in {t_par:.1f} s", file=sys.stderr, flush=True)
    return {"workload": wl.name, "nrhs": wl.nrhs, "n_points": wl.n_points, "J": g.J,
            "t_assemble_s": t_asm, "t_factor_all_s": t_fac, "t_one_rhs_s": t_one, "iters_rhs0": r0.iters,
            "relres_rhs0": r0.relres, "cores": C if t_par else 1, "t_wall_C_rhs_s": t_par,
            "iters_C_rhs": it_par, "sample_strips": list(SAMPLE_STRIPS), "sample_factor_s": t_sfac,
            "sample_solve_s": t_ssol, "host_cpus": os.cpu_count(), "wall_s": time.time() - t0}


def _job_values(rec, scale=1.0):
    """Right-hand sides x points per second of the recorded oracle job (times x scale): one
    core (solves one after another) and C cores (C solves at a time)."""
    t_common = (rec["t_assemble_s"] + rec["t_factor_all_s"]) * scale
    job1 = t_common + rec["nrhs"] * rec["t_one_rhs_s"] * scale
    out = {"one_core": {"value": rec["nrhs"] * rec["n_points"] / job1, "cores": 1, "est_job_s": job1}}
    if rec.get("t_wall_C_rhs_s"):
        C = rec["cores"]
        jobc = t_common + math.ceil(rec["nrhs"] / C) * rec["t_wall_C_rhs_s"] * scale
        out["all_cores"] = {"value": rec["nrhs"] * rec["n_points"] / jobc, "cores": C, "est_job_s": jobc}
    return out


def oracle_record_path(wl):
    return os.path.join(ROOT, "profiles", f"oracle_job_{wl.name}.md")


def read_oracle_record(path):
    """The JSON block of a recorded oracle job summary (Markdown)."""
    text = open(path).read()
    a = text.index("```json") + len("```json")
    return json.loads(text[a:text.index("```", a)])


def write_oracle_record(path, rec, argv):
    with open(path, "w") as fh:
        fh.write(f"# The CPU oracle's whole job on {rec['workload']}\n\n"
                 f"command: `python {' '.join(argv)}` (host of the GPU box, {rec['host_cpus']} CPUs visible)\n\n"
                 "Assembly of the global operator, SuperLU factorisation of every strip, reduced DD-GMRES "
                 "to 1e-6 on right-hand side 0 (one process), then one right-hand side per forked process "
                 "on `cores` processes.  `sample_*`: the bounded sample the default bench run re-times.\n\n"
                 "```json\n" + json.dumps(rec, indent=1) + "\n```\n")


def cpu_baseline(wl, mode):
    """cpu_baseline of the bench line.  mode "full": the oracle's whole job now (several
    minutes at 2000^2).  mode "sample": a bounded sample (SuperLU factorisation and solves of
    SAMPLE_STRIPS, about 10 s) re-timed now, and the committed record of the whole oracle job
    on this workload (profiles/oracle_job_<workload>.md, written by --cpu-baseline full on
    the same kind of host) scaled by the ratio of the sample's time now to the same sample's
    time in the record."""
    if mode == "full":
        rec = oracle_job(wl)
        vals = _job_values(rec)
        best = vals.get("all_cores", vals["one_core"])
        return dict(value=best["value"], unit="RHS*gridpts/s", cores=best["cores"], kind="oracle",
                    sample=(f"the oracle's whole job on {wl.name}, measured now: assembly, SuperLU factorisation "
                            f"of all {rec['J']} strips, reduced DD-GMRES to 1e-6 on right-hand side 0 end to end "
                            f"({rec['iters_rhs0']} iterations, 1 core), then right-hand sides 1..{rec['cores']} on "
                            f"{rec['cores']} forked processes; scaled to {rec['nrhs']} right-hand sides"),
                    **vals, record=rec)
    path = oracle_record_path(wl)
    t0 = time.time()
    from oracle.grid import geometry_from_workload
    g = geometry_from_workload(wl)
    t_sfac, t_ssol = _strip_pieces(g, g.k2(), SAMPLE_STRIPS)
    if not os.path.exists(path):
        return {"value": None, "unit": "RHS*gridpts/s", "cores": 1, "kind": "oracle",
                "sample": f"no record of the oracle's whole job on {wl.name} ({path} missing)"}
    rec = read_oracle_record(path)
    scale = (t_sfac + 2 * t_ssol) / (rec["sample_factor_s"] + 2 * rec["sample_solve_s"])
    vals = _job_values(rec, scale)
    best = vals.get("all_cores", vals["one_core"])
    return dict(value=best["value"], unit="RHS*gridpts/s", cores=best["cores"], kind="oracle",
                sample=(f"SuperLU factorisation and 2 solves of strips {list(SAMPLE_STRIPS)} of {wl.name} re-timed "
                        f"now ({time.time() - t0:.1f} s; {scale:.2f}x their time in the record), scaling the "
                        f"recorded whole oracle job: assembly, all {rec['J']} strip factorisations, reduced "
                        f"DD-GMRES on right-hand side 0 ({rec['iters_rhs0']} iterations, 1 core) and right-hand "
                        f"sides 1..{rec['cores']} on {rec['cores']} processes, scaled to {rec['nrhs']} right-hand "
                        f"sides"),
                **vals, host_scale=scale)


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
                  pml_iface_s0=wl.pml_iface_s0,
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


LENS_CHUNKS = (8, 12, 16, 24, 32)
BATCH_CHUNKS = (16, 24, 32)


def lens_leg(tol, reps=2):
    """The 1000^2 Gaussian-lens workload (16 sources, J = 32), a medium that varies with x
    (every strip has its own factorisation), in complex64-mixed and complex128: factor and
    solve times (mean of `reps` timed passes after one untimed pass) and iteration counts."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1208_3956_amd import Helmholtz
    wl = W.lens_1000()
    f = torch.from_numpy(wl.rhs()).to("cuda:0")
    out = {"workload": wl.name, "nrhs": f.shape[0], "J": wl.J}
    for prec in ("mixed", "c128"):
        H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                      pml_iface_s0=wl.pml_iface_s0, prec=prec, mode="reduced", device="cuda:0")
        # 16 right-hand sides fill one right-hand-side group of the strip kernels, so more,
        # smaller chunks keep more CUs busy: each precision factors with its fastest size
        tuned = H.autotune(f, candidates=LENS_CHUNKS, reps=2, cache=None)
        res = H.solve(f, tol)
        torch.cuda.synchronize()
        tf = ts = 0.0
        for _ in range(reps):
            ta = time.perf_counter()
            H.factor()
            torch.cuda.synchronize()
            tb = time.perf_counter()
            res = H.solve(f, tol)
            torch.cuda.synchronize()
            tf += tb - ta
            ts += time.perf_counter() - tb
        slots = H.factor_slots
        H.close()
        ms = (tf + ts) / reps * 1e3
        out[prec] = {"ms_per_step": ms, "factor_ms": tf / reps * 1e3, "solve_ms": ts / reps * 1e3,
                     "value": f.shape[0] * wl.n_points / (ms / 1e3), "factor_slots": slots,
                     "chunk_rows": tuned["chunk_rows"],
                     "iters": {"min": min(res.iters), "max": max(res.iters),
                               "mean": float(np.mean(res.iters))},
                     "relres_max": max(res.relres)}
        print(f"# lens {prec}: {ms:.0f} ms per step, iterations {sorted(set(res.iters))}",
              file=sys.stderr, flush=True)
    out["mixed_vs_c128"] = out["mixed"]["value"] / out["c128"]["value"]
    return out


def smooth3d_leg(tol, reps=1):
    """The 80^3 smooth 3-D medium (32 sources, 16 slabs), complex64-mixed, reduced: factor
    and solve times of `reps` timed steps after one untimed one, iterations, and the
    complex64 slab factorisation's rate against the FP32 MFMA peak (algorithmic flops of
    phase_flops: B^3 complex multiply-adds per plane of every stored slab factorisation)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1208_3956_amd import Helmholtz
    wl = W.smooth_3d()
    f = torch.from_numpy(wl.rhs()).to("cuda:0")
    H = Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                  pml_iface_s0=wl.pml_iface_s0, prec="mixed", mode="reduced", device="cuda:0")
    H.factor()
    res = H.solve(f, tol)
    torch.cuda.synchronize()
    tf = ts = 0.0
    for _ in range(reps):
        ta = time.perf_counter()
        H.factor()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        res = H.solve(f, tol)
        torch.cuda.synchronize()
        tf += tb - ta
        ts += time.perf_counter() - tb
    slots, path = H.factor_slots, H.factor_path
    fflops = phase_flops(H, wl, f.shape[0])["factor_chunks"]
    H.close()
    ms = (tf + ts) / reps * 1e3
    out = {"workload": wl.name, "nrhs": f.shape[0], "J": wl.J, "ms_per_step": ms,
           "factor_ms": tf / reps * 1e3, "solve_ms": ts / reps * 1e3,
           "value": f.shape[0] * wl.n_points / (ms / 1e3), "factor_slots": slots, "factor_path": path,
           "factor_tflops": fflops / (tf / reps) / 1e12, "factor_frac_fp32_peak": fflops / (tf / reps) / 1e12 / PEAK["c64"],
           "iters": {"min": min(res.iters), "max": max(res.iters), "mean": float(np.mean(res.iters))},
           "relres_max": max(res.relres)}
    print(f"# smooth 3-D: {ms:.0f} ms per step (factor {out['factor_ms']:.0f} ms), iterations "
          f"{sorted(set(res.iters))}", file=sys.stderr, flush=True)
    return out


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
                    pml_iface_s0=wl.pml_iface_s0,
                    prec=args.prec, mode=args.mode, chunk=args.chunk, device=dev, stream=s)
          for wl, s in zip(wls, streams)]
    # the same problems with their strip solves fused into multi-problem launches
    Hf = [Helmholtz(wl.c, wl.omega, wl.h, wl.J, wl.w_out, wl.w, wl.pml_power, wl.pml_s0,
                    pml_iface_s0=wl.pml_iface_s0, prec=args.prec, mode=args.mode, chunk=args.chunk,
                    device=dev, stream=torch.cuda.Stream(dev), batch_fuse=True) for wl in wls]
    pts = sum(f.shape[0] * wl.n_x * wl.n_y for wl, f in zip(wls, fs))
    tuned = None
    if args.chunk == 0:
        # 8 right-hand sides per problem: each handle factors with the chunk size the
        # autotuner finds fastest for it (before the timed steps), among sizes of 16 rows or
        # more: timed alone 8-row chunks win, but eight problems at once then run more and
        # longer separator chains (measured: 534 ms per step with 8 rows, 486 with 16)
        tuned = [H.autotune(f, candidates=BATCH_CHUNKS, reps=1, cache=None)["chunk_rows"]
                 for H, f in zip(Hs, fs)]
        for H, f in zip(Hf, fs):
            H.autotune(f, candidates=BATCH_CHUNKS, reps=1, cache=None)

    solo_ms = [0.0] * len(Hs)

    def step(concurrent):
        if concurrent:
            for H in Hs:
                H.factor()
            for H in Hs:
                H.stream.synchronize()
            return solve_batch(Hs, fs, args.tol)
        # one problem after another, each timed alone (factor + solve)
        out = []
        for k, (H, f) in enumerate(zip(Hs, fs)):
            ta = time.perf_counter()
            H.factor()
            out.append(H.solve(f, args.tol))
            H.stream.synchronize()
            solo_ms[k] += (time.perf_counter() - ta) * 1e3
        return out

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
    solo = [v / (args.steps + args.warmup) for v in solo_ms]

    def step_fused():
        for H in Hf:
            H.factor()
        for H in Hf:
            H.stream.synchronize()
        return solve_batch(Hf, fs, args.tol)

    for k in range(args.warmup):
        step_fused()
    torch.cuda.synchronize()
    print("# batch timed: fused", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res_f = step_fused()
    torch.cuda.synchronize()
    t_f = (time.perf_counter() - t0) / args.steps
    for H in Hs + Hf:
        H.close()
    out = {
        "metric": "RHS*gridpts/s to 1e-6 residual, uneven batch of 8 layered 2-D problems (500^2..2000^2, 8 RHS each)",
        "value": pts / t_b, "unit": "RHS*gridpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_b * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64" if args.prec == "mixed" else "c128", "data": "synthetic",
        "config": {"workload": "layers_uneven_batch", "sizes": [wl.n_x for wl in wls],
                   "J": [wl.J for wl in wls], "nrhs_each": 8, "prec": args.prec, "mode": args.mode,
                   "step": "helm_factor (each) + helm_solve_batch",
                   "chunk_rows": tuned if tuned is not None else args.chunk},
        "sequential_value": pts / t_s, "sequential_ms_per_step": t_s * 1e3,
        # each problem's factor + solve alone; the concurrent step cannot be shorter than the
        # slowest of them (the dependency chain of its sweeps and iterations)
        "alone_ms_per_problem": solo, "slowest_alone_ms": max(solo),
        "concurrent_over_slowest_alone": t_b * 1e3 / max(solo),
        # strip solves fused into multi-problem launches (batch_fuse), lockstep rounds
        "fused_value": pts / t_f, "fused_ms_per_step": t_f * 1e3,
        "fused_launches": res_f[0].fused_launches, "unfused_launches": res_f[0].unfused_launches,
        "iters": [float(np.mean(r.iters)) for r in res],
        "relres_max": max(max(r.relres) for r in res + res_s + res_f),
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
                  pml_iface_s0=wl.pml_iface_s0, sweep=args.sweep,
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
    # timed steps: the configured path as a user runs it (reduced operator replayed from its
    # HIP graph, no event timing)
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
    ms_step = (t1 - t0) * 1e3 / args.steps
    # breakdown step: every hot-kernel class timed with HIP events (kernel by kernel: the
    # durations of events inside a graph replay cannot be read), names the dominant class
    H.set_kernel_timing(True)
    H.factor()
    H.solve(f, args.tol)
    torch.cuda.synchronize()
    kt_all = H.kernel_times()
    dom = max(PHASES, key=lambda k: kt_all[k][1])
    # launch duration of the dominant class: further steps with only that class bracketed by
    # events on the solver's stream, the rest undisturbed
    H.set_kernel_timing(True, classes=[dom])
    for k in range(args.roofline_steps):
        H.factor()
        H.solve(f, args.tol)
    torch.cuda.synchronize()
    kt = H.kernel_times()
    H.set_kernel_timing(False)
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
            "launches": cnt, "avg_launch_us": avg_s * 1e6, "flops_per_launch": fl[dom],
            "avg_launch_from": (f"HIP events around every {dom} launch on the solver's stream during "
                                f"{args.roofline_steps} steps run after the timed ones (same inputs and "
                                "kernels, reduced operator launched kernel by kernel)")}
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
                   "factor_slots": H.factor_slots, "pml_iface_s0": wl.pml_iface_s0 if wl.pml_iface_s0 is not None else "2.5 per pad cell",
                   "graph_replay": args.mode == "reduced", "sweep": args.sweep,
                   "step": "helm_factor + helm_solve"},
        "solve_only_value": pts / (solve_ms / 1e3), "solve_ms": solve_ms,
        "factor_ms": t_fac * 1e3 / args.steps,
        "iters": {"min": min(res.iters), "max": max(res.iters),
                  "mean": float(np.mean(res.iters))},
        "relres_max": max(res.relres), "restarts": res.restarts,
        "preconditioner_applications": res.ap_applies,
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
    if wl.dim == 2 and wl.name.startswith("layers") and not args.no_lens_leg:
        out["lens_1000"] = lens_leg(args.tol)
    if wl.dim == 2 and wl.name.startswith("layers") and not args.no_3d_leg:
        out["smooth_3d"] = smooth3d_leg(args.tol)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_baseline)
        if args.cpu_baseline == "full" and args.oracle_record_out:
            write_oracle_record(args.oracle_record_out, out["cpu_baseline"]["record"], sys.argv)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
