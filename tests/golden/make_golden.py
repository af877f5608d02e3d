"""Write the stored oracle results used by the full-size parity tests and the
benchmark's accuracy check.  Calls only the CPU FP64 oracle (oracle/) on
inputs from the seeded generators (workloads/); nothing here comes from the
GPU library.

python tests/golden/make_golden.py [name ...]     (default: every case)

Each case writes tests/golden/<name>.json with the input's content digest,
the parameters, the per-run values and the assembled estimate.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

# name -> (matrix builder, method, n_probes, sketch_rank, krylov_steps, iop_window, seed, hints)
CASES = {
    "lap3d128_s1e-2_oslq_k2": (lambda: W.lap3d(128, 1e-2), "oslq", 96, 32, 50, 2, 0, (0.0, 0.0)),
    "lap3d128_s1e-3_oslq_k2": (lambda: W.lap3d(128, 1e-3), "oslq", 96, 32, 50, 2, 0, (0.0, 0.0)),
    "lap3d128_s1e-2_oslq_k8": (lambda: W.lap3d(128, 1e-2), "oslq", 96, 32, 50, 8, 0, (0.0, 0.0)),
    "lap3d128_s1e-2_osaiop_k2": (lambda: W.lap3d(128, 1e-2), "osa_iop", 96, 32, 50, 2, 0, (0.0, 0.0)),
    "er1e6_oslq_k4": (lambda: W.er_laplacian(1_000_000, 8_000_000, seed=0, shift=0.05), "oslq",
                      128, 42, 60, 4, 0, (0.0, 0.0)),
    "wendland5e5_oslq_k2": (lambda: W.wendland(500_000, 48.0, 1e-2, seed=0), "oslq", 64, 21, 40, 2,
                            0, (1e-2, 0.0)),
    # the rest of the 128^3 grid: shift 1e-1, windows 4 and 8, both methods
    "lap3d128_s1e-1_oslq_k2": (lambda: W.lap3d(128, 1e-1), "oslq", 96, 32, 50, 2, 0, (0.0, 0.0)),
    "lap3d128_s1e-1_osaiop_k2": (lambda: W.lap3d(128, 1e-1), "osa_iop", 96, 32, 50, 2, 0,
                                 (0.0, 0.0)),
    "lap3d128_s1e-2_oslq_k4": (lambda: W.lap3d(128, 1e-2), "oslq", 96, 32, 50, 4, 0, (0.0, 0.0)),
    "lap3d128_s1e-2_osaiop_k4": (lambda: W.lap3d(128, 1e-2), "osa_iop", 96, 32, 50, 4, 0,
                                 (0.0, 0.0)),
    "lap3d128_s1e-2_osaiop_k8": (lambda: W.lap3d(128, 1e-2), "osa_iop", 96, 32, 50, 8, 0,
                                 (0.0, 0.0)),
    # the Wendland covariance with its values rounded to bfloat16: the FP64
    # reference of the matrix a bfloat16-valued product actually multiplies
    "wendland5e5_bf16_oslq_k2": (lambda: W.round_values_bf16(W.wendland(500_000, 48.0, 1e-2, seed=0)),
                                 "oslq", 64, 21, 40, 2, 0, (1e-2, 0.0)),
}


def run_case(name: str) -> dict:
    build, method, npr, s, m, k, seed, (lo, hi) = CASES[name]
    t0 = time.time()
    a = build()
    t1 = time.time()
    fn = oracle.oslq if method == "oslq" else oracle.osa_iop
    res = fn(a, npr, s, m, k, seed, lo_hint=lo, hi_hint=hi)
    t2 = time.time()
    return {
        "name": name, "matrix": a.name, "n": a.n, "nnz": a.nnz, "digest": W.csr_digest(a),
        "method": method, "n_probes": npr, "sketch_rank": s, "krylov_steps": m,
        "iop_window": k, "seed": seed, "lo_hint": lo, "hi_hint": hi,
        "logdet": res.logdet, "tr_sketch": res.tr_sketch, "tr_resid": res.tr_resid,
        "shift_c": res.shift_c, "lambda_lo": res.lambda_lo, "lambda_hi": res.lambda_hi,
        "scale": res.scale, "probe_K": res.probe_K, "probe_norm2": res.probe_norm2,
        "probe_steps": res.probe_steps, "oracle_seconds": t2 - t1, "build_seconds": t1 - t0,
    }


def main(argv):
    names = argv or list(CASES)
    for name in names:
        out = os.path.join(HERE, name + ".json")
        print(f"[golden] {name} ...", flush=True)
        rec = run_case(name)
        with open(out, "w") as f:
            json.dump(rec, f, indent=1)
        print(f"[golden] {name}: logdet {rec['logdet']!r} in {rec['oracle_seconds']:.1f} s",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
