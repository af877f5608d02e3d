#!/usr/bin/env python3
"""Throughput benchmark of the OSLQ / OSA-IOP hot path on one MI355X.

A step is one whole log-determinant estimate (probe generation, sketch
product, CholQR2, projection, every Krylov step of every run, quadrature and
trace assembly) on a 3D 7-point Laplacian of 128^3 unknowns plus 1e-2 I,
96 Rademacher probes (sketch 32 + 64 residual), 50 Krylov steps, window 2,
seed 0.  The matrix is resident in device memory before the clock starts.

Prints one JSON line: probe-steps/s (one Krylov run advancing one step is
one probe-step), the roofline of the dominant kernel family measured with HIP
events on the library's stream over the timed steps (the family is named by
one untimed estimate with every family timed, which also gives the per-family
device times reported as kernel_families), the accuracy of the
timed configuration against the FP64 path and the stored FP64 oracle
result, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s

FAMILIES = ("spmm", "dots", "update", "reduce", "small", "sketch", "probes")


PRECISIONS = {"mixed": lambda L: L.LD_PREC_MIXED, "half": lambda L: L.LD_PREC_HALF,
              "fp64": lambda L: L.LD_PREC_FP64, "auto": lambda L: L.LD_PREC_AUTO}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--method", choices=("oslq", "osa_iop"), default="oslq")
    ap.add_argument("--precision", choices=("mixed", "half", "fp64"), default="mixed",
                    help="Krylov vectors in FP32 (mixed: FP32 vectors and values, FP64 "
                         "reductions and small matrices), FP16 (half) or FP64")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other full-size configurations (graph, Wendland)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip timing the other precisions on the headline workload")
    ap.add_argument("--values", choices=("fp32", "bf16"), default="fp32")
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--shift", type=float, default=1e-2)
    ap.add_argument("--probes", type=int, default=96)
    ap.add_argument("--sketch", type=int, default=32)
    ap.add_argument("--krylov-steps", type=int, default=50)
    ap.add_argument("--window", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--cpu-probes", type=int, default=12)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-nmax", type=float, default=2e6)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--copy-bytes", type=float, default=805306368,
                    help="bytes of the copy-kernel calibration (0 to skip)")
    ap.add_argument("--no-comparators", action="store_true",
                    help="skip the SLQ / So-SLQ / adaptive / OSA-IOP leg on the same matrix")
    ap.add_argument("--no-grf", action="store_true",
                    help="skip the GRF likelihood theta-sweep leg")
    ap.add_argument("--grf-grid", type=str, default="900x1200")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the kernel-by-kernel vs graph-replay leg")
    ap.add_argument("--tune-reps", type=int, default=10,
                    help="launches per candidate of the product/update geometry autotuner "
                         "(0 keeps the default geometry)")
    ap.add_argument("--config-geometry", action="append", default=[],
                    help="NAME=L,C,E,I[,S][+rg]/L,C[/P]: pin the FP32-vector geometry of a "
                         "full-size configuration leg instead of autotuning it (repeatable)")
    ap.add_argument("--geometry", type=str, default=None,
                    help="pin the headline geometry instead of autotuning it: "
                         "'L,C,E,I[,S][+rg]/L,C[/P]' = product lanes per row, chunks per lane, "
                         "entry split, interleave[, row-tile stride][, row groups] / update "
                         "lanes per row, "
                         "chunks per lane [/ step schedule: 1 the product subtracts the "
                         "second-newest window vector (default), 0 the update]")
    return ap.parse_args()


def parse_geometry(spec):
    parts = spec.split("/")
    prod = parts[0]
    rg = prod.endswith("+rg")
    pv = [int(x) for x in prod[:-3 if rg else None].split(",")]
    pl, pc, pe, pi = pv[:4]
    ps = pv[4] if len(pv) > 4 else 0
    ul, uc = (int(x) for x in parts[1].split(","))
    sched = int(parts[2]) if len(parts) > 2 else 1
    return {"spmm_lanes": pl, "spmm_chunks": pc, "spmm_entry_split": pe, "spmm_interleave": pi,
            "spmm_row_stride": ps, "spmm_row_groups": int(rg), "update_lanes": ul,
            "update_chunks": uc, "step_presub": sched, "pinned": True}


def set_geometry(L, h, p, tune):
    L.ld_tune_set(h, p, tune["spmm_lanes"], tune["spmm_chunks"], tune["update_lanes"],
                  tune["update_chunks"], spmm_entry_split=tune["spmm_entry_split"],
                  spmm_interleave=tune["spmm_interleave"],
                  spmm_row_stride=tune.get("spmm_row_stride", 0),
                  step_presub=tune.get("step_presub", 1),
                  spmm_row_groups=tune.get("spmm_row_groups", 0))


def geometry_key(tune):
    """The geometry a PMC record was taken with: 'default', or the product's
    'L,C,E,I' (lanes, chunks, entry split, interleave), with ',S' when its
    rows are taken in tiles of stride S, '+rg' when it reads the matrix's row
    groups and '+plain' when the update, not the product, subtracts the
    second-newest window vector."""
    if not tune:
        return "default"
    key = (f"{tune['spmm_lanes']},{tune['spmm_chunks']},{tune['spmm_entry_split']},"
           f"{tune['spmm_interleave']}")
    if tune.get("spmm_row_stride", 0):
        key += f",{tune['spmm_row_stride']}"
    if tune.get("spmm_row_groups", 0):
        key += "+rg"
    if not tune.get("step_presub", 1):
        key += "+plain"
    return key


def pmc_record(key):
    """The committed PMC record of a workload key, or None when there is none
    or the kernel source changed since its counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        db = json.load(f)
    recs = [r for r in db.get("records", []) if r.get("workload") == key]
    if not recs:
        return None
    for src, digest in recs[0].get("sources", {}).items():
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return recs[0]


def pmc_traffic(args, family, tune):
    """HBM bytes per launch of `family`'s kernel from the committed PMC summary.

    FETCH_SIZE and WRITE_SIZE were taken with rocprofv3 on this workload and
    scaled by what they read for a plain copy of known size.  The kernel
    instance is the one of the geometry this run used (its chunks-per-lane
    template argument).  Returns None when the workload differs, the kernel
    source changed since the counters were taken, or that instance was not
    profiled (the figures would then describe another kernel).
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        db = json.load(f)
    key = (f"{args.method} {args.precision} values={args.values} lap3d {args.grid} "
           f"shift={args.shift:g} probes={args.probes} sketch={args.sketch} "
           f"m={args.krylov_steps} k={args.window} seed={args.seed}")
    recs = [r for r in db.get("records", []) if r.get("workload") == key]
    if not recs:
        return None
    rec = recs[0]
    for src, digest in rec.get("sources", {}).items():
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    pattern = rec.get("family_kernel", {}).get(family)
    if pattern is None:
        return None
    if tune:
        chunks = tune["spmm_chunks"] if family == "spmm" else tune["update_chunks"]
        split = tune.get("spmm_entry_split", 1) > 1
    else:
        chunks = rec.get("default_chunks", {}).get(family)
        split = False
    kname = pattern.replace("{C}", str(chunks)).replace("{S}", "true" if split else "false")
    # the product's traffic depends on its whole geometry (lanes, chunks,
    # split, chunk mapping): only counters taken with this run's geometry
    # count; the update streams every block once whatever its lanes
    geo = geometry_key(tune)
    tables = rec.get("geometries", {})
    if family == "spmm":
        k = tables.get(geo, {}).get(kname)
    else:
        k = next((t[kname] for t in tables.values() if kname in t), None)
    if k is None:
        return None
    return {"bytes_per_launch": k["scaled_bytes"], "kernel": kname, "geometry": geo,
            "fetch_scale": rec["fetch_scale"], "write_scale": rec["write_scale"],
            "summary": rec.get("summary")}


def stream_ceiling(L, ctx, nbytes):
    """Attainable streaming bandwidth on this GPU at several read:write mixes
    (the library's plain streaming kernel, 16 bytes per lane): the ceiling a
    kernel with the same mix can reach, beside the 8 TB/s published peak."""
    out = {}
    for reads, writes in ((1, 0), (2, 0), (1, 1), (2, 1), (3, 1)):
        ms = L.ld_debug_stream(ctx.handle, nbytes, reads, writes, 10)
        out[f"{reads}r{writes}w"] = {"ms": ms,
                                     "GB/s": (reads + writes) * nbytes / (ms * 1e-3) / 1e9}
    print(f"[bench] stream ceiling {out}", file=sys.stderr, flush=True)
    return out


def golden_for(matrix_name, args):
    """The stored oracle result (tests/golden/*.json) for this exact matrix,
    method and parameters, if one was recorded."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "tests", "golden", "*.json")):
        with open(path) as f:
            g = json.load(f)
        if (g.get("matrix") == matrix_name and g.get("method") == args.method
                and g.get("n_probes") == args.probes and g.get("sketch_rank") == args.sketch
                and g.get("krylov_steps") == args.krylov_steps
                and g.get("iop_window") == args.window and g.get("seed") == args.seed):
            return g
    return None


def golden_file(name):
    """The stored oracle result tests/golden/<name>.json, if present."""
    path = os.path.join(ROOT, "tests", "golden", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def host_cpu():
    """Host CPU model and the logical CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - not Linux
        avail = os.cpu_count()
    return {"model": model, "nproc": avail, "os_cpu_count": os.cpu_count()}


def cpu_baseline(a, args):
    """The CPU FP64 oracle, as it stands, on a bounded sample of the same
    workload: the same matrix and Krylov settings, fewer probes."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover - threadpoolctl missing
        limiter = None
    npr = max(2, args.cpu_probes)
    s = max(1, npr // 3)
    fn = oracle.oslq if args.method == "oslq" else oracle.osa_iop
    t0 = time.perf_counter()
    res = fn(a, npr, s, args.krylov_steps, args.window, args.seed)
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    steps = sum(res.probe_steps) + (args.krylov_steps * s if args.method == "osa_iop" else 0)
    return {"value": steps / dt, "unit": "probe-steps/s", "cores": 1, "kind": "oracle",
            "host": host_cpu(),
            "threads": "one: BLAS limited to 1 thread, scipy.sparse products single-threaded",
            "sample": f"{args.method} oracle, same {a.name} matrix, {npr} probes "
                      f"(sketch {s}), {args.krylov_steps} steps, window {args.window}: "
                      f"{steps} probe-steps in {dt:.1f} s"}


def comparators_bench(L, W, ctx, h, a, vt, args):
    """The paper's comparison (SLQ, So-SLQ, OSLQ, OSA-IOP, Section 4) redone on
    the benchmark matrix: one estimate each after a warm-up, the same total
    probe count, mixed precision; error against the closed form.  So-SLQ and
    OSA-IOP also run Krylov blocks of the sketch width, which the headline's
    autotuning pass does not cover: they get a pass of their own."""
    exact = W.lap3d_exact_logdet(args.grid, args.shift) if args.grid in (64, 128) else None
    npr, m, win = args.probes, args.krylov_steps, args.window
    cases = {
        "slq": L.make_params(npr, 0, m, win, args.seed),
        "oslq": L.make_params(npr, args.sketch, m, win, args.seed),
        "oslq_adaptive_1e-6": L.make_params(npr, args.sketch, m, win, args.seed, adapt_tol=1e-6,
                                             adapt_every=5),
        "so_slq_q30_k10": L.make_params(30 + (npr - args.sketch), 30, m, win, args.seed,
                                        method=L.LD_METHOD_SO_SLQ, subspace_rank=10,
                                        probe_dist=L.LD_PROBE_GAUSSIAN),
        "osa_iop": L.make_params(npr, args.sketch, m, win, args.seed,
                                 method=L.LD_METHOD_OSA_IOP),
    }
    out = {}
    for name, p in cases.items():
        p.precision = PRECISIONS[args.precision](L)
        if args.tune_reps > 0 and name in ("so_slq_q30_k10", "osa_iop"):
            L.ld_autotune(h, p, args.tune_reps)
        L.ld_estimate_ex(h, p)
        t0 = time.perf_counter()
        r = L.ld_estimate_ex(h, p)
        dt = time.perf_counter() - t0
        rec = {"logdet": r.logdet, "ms": dt * 1e3, "device_ms": r.device_ms,
               "probe_steps": r.probe_steps, "probe_steps_per_s": r.probe_steps / dt,
               "matvecs": r.matvecs, "min_steps": r.min_steps}
        if exact:
            rec["rel_err_vs_closed_form"] = abs(r.logdet - exact) / abs(exact)
        out[name] = rec
        print(f"[bench] comparator {name} {rec}", file=sys.stderr, flush=True)
    return out


def grf_bench(L, W, args):
    """GRF likelihood sweep (Section 4): the seven theta candidates on the
    900 x 1200 grid, Wendland covariance with support radius theta/10 grid
    spacings and nugget 1e-2, all requests in flight together; the paper's
    settings for each estimator (OSLQ: 60 steps, 30 probes; OSA-IOP: 20
    steps, 21 probes, tol 1e-6), mixed precision."""
    from paper_2606_07004_amd import grf
    ny, nx = (int(v) for v in args.grf_grid.split("x"))
    x = W.grf_field(ny, nx, seed=11)
    legs = {
        "oslq": L.make_params(30, 10, 60, 2, args.seed, precision=L.LD_PREC_MIXED),
        "osa_iop": L.make_params(21, 7, 20, 2, args.seed, method=L.LD_METHOD_OSA_IOP,
                                 precision=L.LD_PREC_MIXED, tol=1e-6),
    }
    cache = {}

    def make(th):
        if th not in cache:
            cache[th] = W.wendland_grid(ny, nx, W.grf_rho(th), nugget=1e-2)
        return cache[th]

    t0 = time.perf_counter()
    for th in W.GRF_THETAS:
        make(th)
    build_s = time.perf_counter() - t0
    out = {"grid": f"{ny}x{nx}", "n": ny * nx, "thetas": list(W.GRF_THETAS),
           "nnz": [cache[th].nnz for th in W.GRF_THETAS], "host_build_s": build_s}
    with L.Context(0, max_slots=8) as c:
        for name, p in legs.items():
            recs = grf.theta_sweep(c, W.GRF_THETAS, make, x, p, lo_hint=lambda th: 1e-2,
                                   vt=L.LD_VT_FP32)
            out[name] = {"sweep_wall_s": recs[0]["sweep_wall_s"],
                         "logdets_per_s": len(recs) / recs[0]["sweep_wall_s"],
                         "best_theta": grf.best_theta(recs),
                         "logdet": [r["logdet"] for r in recs],
                         "loglik": [r["loglik"] for r in recs],
                         "latency_ms": [r["latency_ms"] for r in recs]}
            print(f"[bench] grf {name} {out[name]}", file=sys.stderr, flush=True)
    return out


def configs_bench(L, W, args):
    """The other full-size configurations of the workload table: the
    Erdos-Renyi graph Laplacian (n = 1e6, 17e6 entries, 128 probes = 42 + 86,
    60 steps, window 4) and the Wendland covariance (n = 5e5, 24.4e6 entries,
    64 probes = 21 + 43, 40 steps, window 2, lower hint 1e-2), FP32 values.
    Per precision: probe-steps/s over a few blocking estimates after a tuning
    pass, and the distance from the stored FP64 oracle result of the same
    seeded inputs.  For FP32 vectors also the product kernel: its time per
    launch and rate on algorithmic bytes (HIP events, one estimate), and on
    the bytes its L2 misses fetch (FETCH_SIZE / WRITE_SIZE from the committed
    PMC record of this configuration, when the kernel source still matches)."""
    out = {}
    cases = {
        "er1e6_oslq_k4": (lambda: W.er_laplacian(1_000_000, 8_000_000, seed=0, shift=0.05),
                          128, 42, 60, 4, 0.0),
        "wendland5e5_oslq_k2": (lambda: W.wendland(500_000, 48.0, 1e-2, seed=0), 64, 21, 40, 2,
                                1e-2),
    }
    pinned = dict(g.split("=", 1) for g in args.config_geometry)
    with L.Context(0) as ctx:
        for name, (build, npr, s, m, k, lo) in cases.items():
            a = build()
            gold = golden_file(name)
            h = ctx.matrix(a, vt=L.LD_VT_FP32, lo_hint=lo)
            rec = {"n": a.n, "nnz": a.nnz, "probes": npr, "sketch": s, "steps": m, "window": k}
            del a
            for prec in ("mixed", "fp64", "half", "auto"):
                p = L.make_params(npr, s, m, k, 0, precision=PRECISIONS[prec](L))
                tune = None
                try:
                    if prec == "mixed" and name in pinned:
                        tune = parse_geometry(pinned[name])
                        set_geometry(L, h, p, tune)
                    elif args.tune_reps > 0 and prec != "auto":
                        tune = L.ld_autotune(h, p, args.tune_reps).as_dict()
                    r = L.ld_estimate_ex(h, p)
                except L.LdError as e:
                    # FP16 vectors are refused outside the range where they
                    # hold 1e-4 (spectral bound ratio above 512, window above 4)
                    rec[prec] = {"refused": str(e)}
                    continue
                reps = 3
                steps = 0
                t0 = time.perf_counter()
                for _ in range(reps):
                    steps += L.ld_estimate_ex(h, p).probe_steps
                dt = time.perf_counter() - t0
                rec[prec] = {"probe_steps_per_s": steps / dt, "ms_per_estimate": dt * 1e3 / reps,
                             "logdet": r.logdet,
                             "rel_err_vs_oracle": (abs(r.logdet - gold["logdet"]) / abs(gold["logdet"])
                                                   if gold else None)}
                if prec == "mixed":
                    L.ld_profile_enable(ctx.handle, L.LD_PROF_SPMM)
                    L.ld_estimate_ex(h, p)
                    n_l, ms, by = L.ld_profile_query(ctx.handle, L.LD_PROF_SPMM)
                    L.ld_profile_enable(ctx.handle, 0)
                    ml = ms / max(1, n_l)
                    prod = {"launches": n_l, "ms_per_launch": ml,
                            "algorithmic_GB": by / max(1, n_l) / 1e9,
                            "algorithmic_GB/s": by / (ms * 1e-3) / 1e9 if ms > 0 else None,
                            "fabric_GB": None, "fabric_GB/s": None}
                    pr = pmc_record(f"config {name} mixed")
                    # the counters describe the product geometry they were
                    # taken with: reported only for the same geometry
                    geo = geometry_key(tune)
                    prod["geometry"] = geo
                    prod["update_geometry"] = (f"{tune['update_lanes']},{tune['update_chunks']}"
                                               if tune else "default")
                    prod["step_presub"] = tune.get("step_presub", 1) if tune else 1
                    prod["interleaved"] = tune["spmm_interleave"] if tune else 0
                    prod["row_groups"] = tune.get("spmm_row_groups", 0) if tune else 0
                    kname = (f"ld::k_spmm_rg<float, float, {tune['spmm_chunks']}, " if prod["row_groups"] else
                             f"ld::k_spmm<float, float, {tune['spmm_chunks'] if tune else 0}, ")
                    ks = [v for kn, v in (pr or {}).get("geometries", {}).get(geo, {}).items()
                          if kn.startswith(kname)]
                    if ks:
                        fb = max(ks, key=lambda v: v["dispatches"])["scaled_bytes"]
                        prod["fabric_GB"] = fb / 1e9
                        prod["fabric_GB/s"] = fb / (ml * 1e-3) / 1e9
                        prod["pmc_summary"] = pr.get("summary")
                    rec[prec]["product"] = prod
            ctx.release(h)
            if name.startswith("wendland"):
                # the same covariance stored with FP64 and BF16 values (FP32
                # Krylov vectors): BF16 rounding changes the matrix, so its
                # distance from the FP64 oracle of the FP64-valued matrix is
                # reported, not gated
                a = build()
                p = L.make_params(npr, s, m, k, 0, precision=L.LD_PREC_MIXED)
                rec["values"] = {"fp32": rec["mixed"]["rel_err_vs_oracle"]}
                for vname, vt in (("fp64", L.LD_VT_FP64), ("bf16", L.LD_VT_BF16)):
                    hv = ctx.matrix(a, vt=vt, lo_hint=lo)
                    L.ld_estimate_ex(hv, p)
                    t0 = time.perf_counter()
                    r = L.ld_estimate_ex(hv, p)
                    dt = time.perf_counter() - t0
                    rec["values"][vname] = abs(r.logdet - gold["logdet"]) / abs(gold["logdet"]) if gold else None
                    rec["values"][vname + "_ms"] = dt * 1e3
                    ctx.release(hv)
                del a
            out[name] = rec
            print(f"[bench] config {name} {rec}", file=sys.stderr, flush=True)
    return out


def window_variants(L, ctx, h, args):
    """The headline matrix with windows 4 and 8 (OSLQ and OSA-IOP): FP32-vector
    probe-steps/s and the distance from the FP64 estimate of the same
    parameters (the headline itself is window 2)."""
    out = {}
    for method, mcode in (("oslq", L.LD_METHOD_OSLQ), ("osa_iop", L.LD_METHOD_OSA_IOP)):
        for k in (4, 8):
            p = L.make_params(args.probes, args.sketch, args.krylov_steps, k, args.seed,
                              method=mcode, precision=L.LD_PREC_MIXED)
            p64 = L.make_params(args.probes, args.sketch, args.krylov_steps, k, args.seed,
                                method=mcode, precision=L.LD_PREC_FP64)
            r64 = L.ld_estimate_ex(h, p64)
            L.ld_estimate_ex(h, p)
            reps = 2
            steps = 0
            t0 = time.perf_counter()
            for _ in range(reps):
                r = L.ld_estimate_ex(h, p)
                steps += r.probe_steps
            dt = time.perf_counter() - t0
            out[f"{method}_k{k}"] = {"probe_steps_per_s": steps / dt,
                                      "ms_per_estimate": dt * 1e3 / reps, "logdet": r.logdet,
                                      "rel_err_vs_fp64_gpu": abs(r.logdet - r64.logdet) / abs(r64.logdet),
                                      "fp64_ms": r64.device_ms}
            print(f"[bench] window {method} k={k} {out[f'{method}_k{k}']}", file=sys.stderr,
                  flush=True)
    return out


def shift_variants(L, W, args):
    """The headline Laplacian with the other shifts of its configuration
    (1e-3 and 1e-1; the headline is 1e-2): FP32 vectors and LD_PREC_AUTO
    (FP64 at 1e-3, where lambda_hi / lambda_lo is 12006), each against the
    FP64 estimate and the closed-form log-determinant, each precision after
    its own autotuning pass on the new matrix (as the headline)."""
    out = {}
    with L.Context(0) as ctx:
        for shift in (1e-3, 1e-1):
            a = W.lap3d(args.grid, shift)
            h = ctx.matrix(a, vt=L.LD_VT_FP32)
            exact = W.lap3d_exact_logdet(args.grid, shift)
            rec = {"closed_form": exact}
            p64 = L.make_params(args.probes, args.sketch, args.krylov_steps, args.window,
                                args.seed, precision=L.LD_PREC_FP64)
            if args.tune_reps > 0:
                L.ld_autotune(h, p64, args.tune_reps)
            r64 = L.ld_estimate_ex(h, p64)
            rec["fp64_ms"] = r64.device_ms
            for name, prec in (("mixed", L.LD_PREC_MIXED), ("auto", L.LD_PREC_AUTO)):
                p = L.make_params(args.probes, args.sketch, args.krylov_steps, args.window,
                                  args.seed, precision=prec)
                if args.tune_reps > 0 and prec == L.LD_PREC_MIXED:
                    L.ld_autotune(h, p, args.tune_reps)
                L.ld_estimate_ex(h, p)
                reps = 2
                t0 = time.perf_counter()
                for _ in range(reps):
                    r = L.ld_estimate_ex(h, p)
                dt = (time.perf_counter() - t0) / reps
                rec[name] = {"ms_per_estimate": dt * 1e3, "probe_steps_per_s": r.probe_steps / dt,
                             "rel_err_vs_fp64_gpu": abs(r.logdet - r64.logdet) / abs(r64.logdet),
                             "rel_err_vs_closed_form": abs(r.logdet - exact) / abs(exact)}
            lo, hi = L.ld_matrix_bounds(h)
            rec["bound_ratio"] = hi / lo
            ctx.release(h)
            out[f"shift_{shift:g}"] = rec
            print(f"[bench] shift {shift:g} {rec}", file=sys.stderr, flush=True)
    return out


def precision_variants(L, ctx, h, args, ref):
    """The headline workload with the Krylov vectors in the other precisions
    (FP32 and FP64 beside FP16): probe-steps/s over a few blocking estimates
    after a tuning pass, and the distance of each from the FP64 result."""
    out = {}
    for name in ("half", "mixed", "fp64"):
        if name == args.precision:
            continue
        p = L.make_params(args.probes, args.sketch, args.krylov_steps, args.window, args.seed,
                          method=L.LD_METHOD_OSLQ if args.method == "oslq" else L.LD_METHOD_OSA_IOP,
                          precision=PRECISIONS[name](L))
        try:
            if args.tune_reps > 0:
                L.ld_autotune(h, p, args.tune_reps)
            r = L.ld_estimate_ex(h, p)
        except L.LdError as e:
            out[name] = {"refused": str(e)}
            print(f"[bench] variant {name} refused: {e}", file=sys.stderr, flush=True)
            continue
        reps = max(1, min(args.steps, 5))
        steps = 0
        t0 = time.perf_counter()
        for _ in range(reps):
            steps += L.ld_estimate_ex(h, p).probe_steps
        dt = time.perf_counter() - t0
        out[name] = {"probe_steps_per_s": steps / dt, "ms_per_estimate": dt * 1e3 / reps,
                     "logdet": r.logdet,
                     "rel_err_vs_fp64_gpu": abs(r.logdet - ref) / abs(ref) if ref else None}
        print(f"[bench] variant {name} {out[name]}", file=sys.stderr, flush=True)
    return out


def graph_bench(L, W, args):
    """Launch overhead of a blocking estimate: kernel by kernel (graph mode
    0) against a replayed HIP graph (mode 1), on 3D Laplacians from n = 1.1e4
    to the headline size, mixed precision, the headline's probes, steps and
    window, a new seed per call (one graph serves every seed).  wall_ms is
    host time per estimate, device_ms the events around it; wall - device is
    what the host adds.  Results of the two modes must be bitwise equal."""
    out = {}
    for grid in (22, 48, 80, args.grid):
        rec = {}
        for mode in (0, 1):
            ctx = L.Context(0)
            try:
                L.ld_graph_mode(ctx.handle, mode)
                a = W.lap3d(grid, args.shift)
                h = ctx.matrix(a, vt=L.LD_VT_FP32)
                rec["n"] = a.n

                def est(seed):
                    return L.ld_estimate_ex(h, L.make_params(
                        args.probes, args.sketch, args.krylov_steps, args.window, seed,
                        precision=L.LD_PREC_MIXED))
                est(1)
                est(2)  # mode 1: captured here
                reps = 30 if a.n < 1e6 else 5
                vals, dev = [], 0.0
                t0 = time.perf_counter()
                for i in range(reps):
                    r = est(10 + i)
                    vals.append(r.logdet)
                    dev += r.device_ms
                wall = (time.perf_counter() - t0) * 1e3 / reps
                st = L.ld_graph_stats_get(ctx.handle)
                rec["graph" if mode else "kernel_by_kernel"] = {
                    "wall_ms": wall, "device_ms": dev / reps, "host_ms": wall - dev / reps,
                    "replays": st.replays, "captures": st.captures, "logdets": vals}
            finally:
                ctx.close()
        rec["bitwise_equal"] = rec["graph"]["logdets"] == rec["kernel_by_kernel"]["logdets"]
        rec["speedup"] = rec["kernel_by_kernel"]["wall_ms"] / rec["graph"]["wall_ms"]
        for k in ("graph", "kernel_by_kernel"):
            del rec[k]["logdets"]
        out[f"lap3d_{grid}"] = rec
        print(f"[bench] graph leg lap3d {grid}: {rec}", file=sys.stderr, flush=True)
    return out


def serving_bench(L, W, args):
    """Served log-determinants (the serving workload): requests of uneven n
    (log-uniform up to 2e6), kind (2D / 3D Laplacian, Wendland covariance),
    shift and Krylov depth, every matrix built and resident before the clock.
    Baseline: plain FP64 estimates one at a time.  Served with continuous
    batching: (i) every request submitted at t = 0 (throughput), with
    LD_PREC_AUTO (FP32 Krylov vectors and FP32 values where lambda_hi <= 4096
    lambda_lo, FP64 beyond: the served form) and with FP32 on every request; (ii)
    Poisson arrivals at 0.7x the FP64 sequential rate, LD_PREC_AUTO (latency
    p50 / p99).  Every served result is compared with its own FP64 result."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    reqs = W.request_stream(args.serve_requests, seed=1, rate_hz=1.0, n_min=1e4,
                            n_max=args.serve_nmax)
    ctx = L.Context(0, max_slots=args.serve_slots)
    try:
        # build on host threads, upload in request order as each finishes (the
        # host copy is dropped after the upload)
        t0 = time.perf_counter()
        hs = [None] * len(reqs)
        nnz = 0
        shapes = [None] * len(reqs)
        with ThreadPoolExecutor(max_workers=8) as ex:
            futs = [ex.submit(W.build_request_matrix, r) for r in reqs]
            for i, (f, r) in enumerate(zip(futs, reqs)):
                a = f.result()
                nnz += a.nnz
                shapes[i] = (a.n, a.nnz)
                # FP64 values plus an FP32 copy: requests with FP32 Krylov
                # vectors read the FP32 values (mixed precision), FP64 ones the
                # FP64 values (LD_PREC_AUTO sends the ill-conditioned requests,
                # nuggets down to 1e-3, to FP64)
                hs[i] = ctx.matrix(a, vt=L.LD_VT_FP32,
                                   lo_hint=(r["shift"] if r["kind"] == "wendland" else 0.0))
                futs[i] = None
                del a
        t_build = time.perf_counter() - t0
        ns = np.array([r["size"] ** {"lap2d": 2, "lap3d": 3}.get(r["kind"], 1) for r in reqs],
                      dtype=np.float64)
        print(f"[bench] serving: built and uploaded {len(reqs)} matrices ({nnz / 1e9:.2f}e9 "
              f"entries) in {t_build:.1f} s", file=sys.stderr, flush=True)

        def params(r, prec):
            return L.make_params(r["n_probes"], r["sketch_rank"], r["krylov_steps"],
                                 r["iop_window"], 1000 + r["id"], precision=prec)
        # warm the kernels once
        L.ld_estimate_ex(hs[0], params(reqs[0], L.LD_PREC_FP64))
        L.ld_estimate_ex(hs[0], params(reqs[0], L.LD_PREC_MIXED))
        t0 = time.perf_counter()
        ref = [L.ld_estimate_ex(h, params(r, L.LD_PREC_FP64)).logdet for h, r in zip(hs, reqs)]
        t_seq = time.perf_counter() - t0
        seq_rate = len(reqs) / t_seq
        print(f"[bench] serving: FP64 sequential {seq_rate:.1f} logdets/s", file=sys.stderr,
              flush=True)
        out = {"requests": len(reqs), "n_range": [1e4, args.serve_nmax],
               "n_median": float(np.median(ns)), "n_max_drawn": float(ns.max()),
               "kinds": {k: sum(1 for r in reqs if r["kind"] == k)
                         for k in ("lap2d", "lap3d", "wendland")},
               "matrix_entries": nnz, "host_build_and_upload_s": t_build,
               "fp64_sequential_logdets_per_s": seq_rate, "slots": args.serve_slots}

        bounds = [L.ld_matrix_bounds(h) for h in hs]

        def alg_bytes(i, res, prec):
            # the request's algorithmic bytes (the per-probe-step model: the
            # matrix once per block of probes, the window vectors read once,
            # the new vector written once); FP32 values with FP32 vectors,
            # FP64 values with FP64 vectors
            n, z = shapes[i]
            r = reqs[i]
            lo, hi = bounds[i]
            fp32 = prec == L.LD_PREC_MIXED or (prec == L.LD_PREC_AUTO and hi <= 4096 * lo)
            sx = 4 if fp32 else 8
            b = r["n_probes"]
            step = (z * (sx + 4) + 4 * (n + 1)) / b + (r["iop_window"] + 1) * n * sx
            return res.probe_steps * step

        def saturate(prec):
            st0 = L.ld_serving_stats_get(ctx.handle)
            t0 = time.perf_counter()
            tickets = [L.ld_submit(h, params(r, prec)) for h, r in zip(hs, reqs)]
            served = [L.ld_wait(ctx.handle, t) for t in tickets]
            dt = time.perf_counter() - t0
            st1 = L.ld_serving_stats_get(ctx.handle)
            errs = [abs(sv.logdet - rf) / abs(rf) for sv, rf in zip(served, ref)]
            tot = sum(alg_bytes(i, sv, prec) for i, sv in enumerate(served))
            return {"logdets_per_s": len(reqs) / dt, "wall_s": dt,
                    "algorithmic_bytes": tot, "algorithmic_GB/s": tot / dt / 1e9,
                    "probe_steps": sum(sv.probe_steps for sv in served),
                    "speedup_vs_fp64_sequential": len(reqs) / dt / seq_rate,
                    "max_rel_err_vs_fp64": max(errs),
                    "requests_over_1e-4": sum(1 for e in errs if e > 1e-4),
                    "batched_launches": st1.batched_launches - st0.batched_launches,
                    "batched_steps": st1.batched_steps - st0.batched_steps}
        ratios = [hi / lo for lo, hi in (L.ld_matrix_bounds(h) for h in hs)]
        out["auto_fp32_requests"] = sum(1 for q in ratios if q <= 4096.0)
        out["served_auto"] = saturate(L.LD_PREC_AUTO)
        print(f"[bench] serving: auto {out['served_auto']}", file=sys.stderr, flush=True)
        out["served_fp32_everywhere"] = saturate(L.LD_PREC_MIXED)
        print(f"[bench] serving: fp32 everywhere {out['served_fp32_everywhere']}",
              file=sys.stderr, flush=True)
        # (ii) Poisson arrivals at 0.7x the FP64 sequential rate, LD_PREC_AUTO
        rate = 0.7 * seq_rate
        rng = np.random.Generator(np.random.PCG64(7))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
        pending = {}
        lat = []
        start = time.perf_counter()
        i = 0
        while i < len(reqs) or pending:
            now = time.perf_counter() - start
            while i < len(reqs) and arrivals[i] <= now:
                pending[L.ld_submit(hs[i], params(reqs[i], L.LD_PREC_AUTO))] = i
                i += 1
            for t in list(pending):
                res = L.ld_poll(ctx.handle, t)
                if res is not None:
                    lat.append(res.latency_ms)
                    del pending[t]
            time.sleep(0.0002)
        lat = np.array(lat)
        st = L.ld_serving_stats_get(ctx.handle)
        out.update({"served_precision": "auto (FP32 Krylov vectors and values where lambda_hi "
                                        "<= 4096 lambda_lo, else FP64)",
                    "served_logdets_per_s": out["served_auto"]["logdets_per_s"],
                    "speedup_vs_fp64_sequential": out["served_auto"]["speedup_vs_fp64_sequential"],
                    "max_rel_err_vs_fp64": out["served_auto"]["max_rel_err_vs_fp64"],
                    "poisson_rate_hz": rate,
                    "p50_latency_ms": float(np.percentile(lat, 50)),
                    "p99_latency_ms": float(np.percentile(lat, 99)),
                    "peak_held_bytes": st.peak_held_bytes, "budget_bytes": st.budget_bytes,
                    "peak_active": st.peak_active})
        for h in hs:
            ctx.release(h)
        return out
    finally:
        ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU "
                                   "layout (probe-parallel runs, one all-gather of the sketch) "
                                   "is designed (see the design notes) but not built"}))
        sys.exit(2)
    import workloads as W
    from paper_2606_07004_amd import liblogdet as L

    t_build = time.perf_counter()
    a = W.lap3d(args.grid, args.shift)
    t_build = time.perf_counter() - t_build
    method = L.LD_METHOD_OSLQ if args.method == "oslq" else L.LD_METHOD_OSA_IOP
    prec = PRECISIONS[args.precision](L)
    vt = L.LD_VT_FP64 if args.precision == "fp64" else (
        L.LD_VT_FP32 if args.values == "fp32" else L.LD_VT_BF16)
    print(f"[bench] {a.name} n={a.n} nnz={a.nnz} built in {t_build:.1f} s", file=sys.stderr,
          flush=True)

    ctx = L.Context(0)
    h = ctx.matrix(a, vt=vt)
    p = L.make_params(args.probes, args.sketch, args.krylov_steps, args.window, args.seed,
                      method=method, precision=prec)

    try:
        L.ld_request_bytes(h, p)  # parameter and precision checks, nothing runs
    except L.LdError as e:
        ctx.close()
        print(json.dumps({"error": f"{args.precision} precision refused on {a.name}: {e}"}))
        sys.exit(2)

    tune = None
    if args.geometry:
        tune = parse_geometry(args.geometry)
        set_geometry(L, h, p, tune)
    elif args.tune_reps > 0:
        t_tune = time.perf_counter()
        tune = L.ld_autotune(h, p, args.tune_reps).as_dict()
        tune["wall_s"] = time.perf_counter() - t_tune
        print(f"[bench] autotune {tune}", file=sys.stderr, flush=True)

    accuracy = {}
    if not args.no_accuracy:
        p64 = L.make_params(args.probes, args.sketch, args.krylov_steps, args.window, args.seed,
                            method=method, precision=L.LD_PREC_FP64)
        r64 = L.ld_estimate_ex(h, p64)
        rt = L.ld_estimate_ex(h, p)
        accuracy["logdet"] = rt.logdet
        accuracy["logdet_fp64_gpu"] = r64.logdet
        accuracy["rel_err_vs_fp64_gpu"] = abs(rt.logdet - r64.logdet) / abs(r64.logdet)
        accuracy["fp64_gpu_ms"] = r64.device_ms
        if args.grid in (64, 128) and args.method == "oslq":
            exact = W.lap3d_exact_logdet(args.grid, args.shift)
            accuracy["closed_form"] = exact
            accuracy["estimator_rel_err_vs_closed_form"] = abs(rt.logdet - exact) / abs(exact)
        gold = golden_for(a.name, args)
        if gold:
            accuracy["oracle_fp64"] = gold["logdet"]
            accuracy["rel_err_fp64_gpu_vs_oracle"] = abs(r64.logdet - gold["logdet"]) / abs(gold["logdet"])
            accuracy["rel_err_vs_oracle"] = abs(rt.logdet - gold["logdet"]) / abs(gold["logdet"])
        print(f"[bench] accuracy {accuracy}", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        L.ld_estimate_ex(h, p)
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    # One untimed estimate with every kernel family bracketed by events gives
    # the per-family device time and names the dominant family; the timed
    # estimates then carry events on that family only (each event pair adds
    # a few microseconds of queue time, ~5% of an estimate for all ~220
    # launches).
    L.ld_profile_enable(ctx.handle, L.LD_PROF_ALL)
    L.ld_estimate_ex(h, p)
    fam = {}
    for name in FAMILIES:
        n, ms, by = L.ld_profile_query(ctx.handle, L.PROF_FAMILIES[name])
        fam[name] = {"launches": n, "ms": ms, "bytes": by}
    dom = max(fam, key=lambda k: fam[k]["ms"])

    L.ld_profile_enable(ctx.handle, L.PROF_FAMILIES[dom])
    total_steps = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = L.ld_estimate_ex(h, p)  # blocking: returns after the device finished
        total_steps += res.probe_steps
    t1 = time.perf_counter()
    elapsed = t1 - t0
    n, ms, by = L.ld_profile_query(ctx.handle, L.PROF_FAMILIES[dom])
    L.ld_profile_enable(ctx.handle, 0)
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    d = {"launches": n, "ms": ms, "bytes": by}
    avg_ms = d["ms"] / max(1, d["launches"])
    bytes_per_launch = d["bytes"] / max(1, d["launches"])
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved * 1e9 / HBM_PEAK, "traffic": None,
                "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": bytes_per_launch}
    tr = pmc_traffic(args, dom, tune)
    if tr is not None:
        roofline["traffic"] = tr["bytes_per_launch"]
        roofline["traffic_detail"] = tr
    # the Krylov step as a whole (product, window dots, update): where the
    # second-newest vector is subtracted moves bytes between the product and
    # the update, not the step's total
    step_fams = ("spmm", "dots", "update")
    st_b = sum(fam[k]["bytes"] for k in step_fams)
    st_ms = sum(fam[k]["ms"] for k in step_fams)
    if st_ms > 0:
        roofline["krylov_step"] = {"families": list(step_fams), "bytes_per_estimate": st_b,
                                   "ms_per_estimate": st_ms,
                                   "achieved": st_b / (st_ms * 1e-3) / 1e9,
                                   "frac": st_b / (st_ms * 1e-3) / HBM_PEAK}
    device_ms_total = sum(v["ms"] for v in fam.values())  # one estimate
    families = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                    "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
                for k, v in fam.items()}

    configs = None
    if not args.no_configs:
        configs = configs_bench(L, W, args)

    variants = None
    windows = None
    shifts = None
    if not args.no_variants:
        variants = precision_variants(L, ctx, h, args, accuracy.get("logdet_fp64_gpu"))
        if args.grid == 128 and args.method == "oslq":
            windows = window_variants(L, ctx, h, args)
            shifts = shift_variants(L, W, args)

    copy = None
    ceiling = None
    if args.copy_bytes > 0:
        nb = int(args.copy_bytes) // 16 * 16
        ms = L.ld_debug_copy(ctx.handle, nb, 10)
        copy = {"bytes": nb, "ms": ms, "GB/s": 2 * nb / (ms * 1e-3) / 1e9}
        print(f"[bench] copy calibration {copy}", file=sys.stderr, flush=True)
        ceiling = stream_ceiling(L, ctx, nb)
        # each Krylov-step kernel against the measured ceiling of its own mix:
        # the product reads two blocks per one written (the gathered input and
        # the window vector it subtracts; the matrix is small beside them), and
        # so does the update at window 2 (the product and the newest vector)
        fam_rate = {k: (v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None)
                    for k, v in fam.items()}
        roofline["kernels"] = {}
        for name, mix in (("spmm", "2r1w"), ("update", "2r1w")):
            rate = achieved if name == dom else fam_rate.get(name)
            if rate:
                roofline["kernels"][name] = {
                    "achieved": rate, "frac_of_peak": rate * 1e9 / HBM_PEAK,
                    "attainable": ceiling[mix]["GB/s"], "attainable_mix": mix,
                    "frac_of_attainable": rate / ceiling[mix]["GB/s"]}

    graphs = None
    if not args.no_graph:
        graphs = graph_bench(L, W, args)

    comparators = None
    if not args.no_comparators:
        comparators = comparators_bench(L, W, ctx, h, a, vt, args)

    serving = None
    if not args.no_serving:
        serving = serving_bench(L, W, args)
        print(f"[bench] serving {serving}", file=sys.stderr, flush=True)

    grf_sweep = None
    if not args.no_grf:
        grf_sweep = grf_bench(L, W, args)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(a, args)
        print(f"[bench] cpu baseline {cpu}", file=sys.stderr, flush=True)

    value = total_steps / elapsed
    out = {
        "metric": "probe-Lanczos steps/s (OSLQ/OSA-IOP Krylov runs advancing one step), "
                  "at rel err <= 1e-4 vs FP64",
        "value": value,
        "unit": "probe-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32", "half": "f16", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.method} 3D 7-point Laplacian {args.grid}^3 + {args.shift:g} I "
                               f"(n={a.n}, nnz={a.nnz}), {args.probes} Rademacher probes "
                               f"(sketch {args.sketch} + {args.probes - args.sketch}), "
                               f"{args.krylov_steps} Krylov steps, window {args.window}, "
                               f"seed {args.seed}",
                   "precision": {"half": "FP16 Krylov vectors, FP32 product sums, FP64 inner "
                                         "products, norms and small matrices",
                                 "mixed": "FP32 Krylov vectors, FP64 inner products, norms and "
                                          "small matrices",
                                 "fp64": "FP64 throughout"}[args.precision],
                   "values": {0: "fp64", 1: "fp32", 2: "bf16"}[vt], "parallelism": "single GPU",
                   "geometry": ({"product": [tune["spmm_lanes"], tune["spmm_chunks"]],
                                 "product_entry_split": tune["spmm_entry_split"],
                                 "product_interleaved": tune["spmm_interleave"],
                                 "product_row_stride": tune.get("spmm_row_stride", 0),
                                 "step_presub": tune.get("step_presub", 1),
                                 "update": [tune["update_lanes"], tune["update_chunks"]]}
                                if tune else "default")},
        "autotune": tune,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "kernel_families": families,
        "serving": serving,
        "graph_replay": graphs,
        "comparators": comparators,
        "precision_variants": variants,
        "window_variants": windows,
        "shift_variants": shifts,
        "configs": configs,
        "grf_sweep": grf_sweep,
        "copy_kernel": copy,
        "stream_ceiling": ceiling,
        "device_ms_per_step": device_ms_total,
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
