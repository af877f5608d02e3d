"""Maximum-likelihood sweep of a Gaussian random field (Section 4).

For each candidate theta the log-likelihood
    L(theta) = log det Q(theta) / 2 - x^T Q(theta) x / 2 - n log(2 pi) / 2
needs one log-determinant; the candidates are independent requests, so they
are queued together with ld_submit and the device works on all of them
(continuous batching), and x^T Q x comes from ld_quad_form.  This module only
orchestrates library calls and assembles the scalars; every product and
estimate runs in the HIP library.
"""
from __future__ import annotations

import math
import time
from typing import Callable, Dict, List, Sequence

from . import liblogdet as L


def theta_sweep(ctx: "L.Context", thetas: Sequence[float], make_matrix: Callable,
                x, params: "L.ld_params", lo_hint: Callable = None,
                vt: int = L.LD_VT_FP64) -> List[Dict]:
    """Submit one estimate per theta, wait for all, return per-theta records
    {theta, n, logdet, quad, loglik, latency_ms, probe_steps}.

    make_matrix(theta) returns a CSR (workloads.Csr-like: n, nnz, row_ptr,
    col_idx, values); lo_hint(theta), when given, is a lower bound of the
    spectrum (for a Wendland covariance, its nugget).  Matrices are created
    one at a time (each host copy can be dropped once on the device) and all
    requests are in flight together."""
    handles, tickets, ns = [], [], []
    t0 = time.perf_counter()
    try:
        for th in thetas:
            a = make_matrix(th)
            h = ctx.matrix(a, vt=vt, lo_hint=lo_hint(th) if lo_hint else 0.0)
            handles.append(h)
            ns.append(a.n)
            del a
            tickets.append(L.ld_submit(h, params))
        results = [L.ld_wait(ctx.handle, t) for t in tickets]
        out = []
        for th, h, n, r in zip(thetas, handles, ns, results):
            q = L.ld_quad_form(h, x)
            out.append({"theta": th, "n": n, "logdet": r.logdet, "quad": q,
                        "loglik": 0.5 * r.logdet - 0.5 * q - 0.5 * n * math.log(2 * math.pi),
                        "latency_ms": r.latency_ms, "probe_steps": r.probe_steps})
        wall = time.perf_counter() - t0
        for rec in out:
            rec["sweep_wall_s"] = wall
        return out
    finally:
        for h in handles:
            ctx.release(h)


def best_theta(records: List[Dict]) -> float:
    """The grid maximiser of the estimated log-likelihood."""
    return max(records, key=lambda r: r["loglik"])["theta"]
