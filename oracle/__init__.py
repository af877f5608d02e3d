"""CPU FP64 oracle for the OSLQ and OSA-IOP log-determinant estimators.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check of the package entry point and the CPU-baseline leg of the
benchmark may import it.  The GPU library never imports, links or calls it,
and it shares no code, tables or constants with the GPU library.

What it follows (Mbingui, Tambue, Karambal, "Optimal Stochastic Krylov Based
Techniques for Large-Scale Log-Determinant Estimation"):

* ``philox``      - Rademacher probes from the Philox4x64-10 counter-based
                    generator (Salmon et al., SC'11); the paper draws +-1 with
                    probability 1/2 (Section 2, eq. (TE); Algs 2 and 3) and
                    names no generator, so both sides implement this one.
                    Gaussian probes (the alternative Section 2 allows) by the
                    Box-Muller transform of the same generator's words.
* ``spectral``    - Gershgorin spectral interval (Section 2.1), the scale
                    gamma = sqrt(lmin lmax) (Proposition 2.1) and the shifts
                    that make the traced operator PSD (eqs. for L in Section
                    2.2 and for J in Section 3.2).
* ``krylov``      - Arnoldi with incomplete orthogonalisation over a window
                    of the last k vectors (Alg 1; window 2 in the paper,
                    k >= m gives full orthogonalisation).
* ``quadrature``  - Gauss quadrature from the tridiagonal T_m (Section 3.1,
                    eq. gauss_quadrature) and log(H_m) e1 (Alg 1, via the
                    principal matrix logarithm).
* ``estimators``  - OSLQ (Alg 3), OSA-IOP (Alg 2), plain Hutchinson/SLQ
                    as the sketch-rank-0 setting, and the So-SLQ comparator of
                    Section 4 (subspace from the dominant left singular
                    vectors of a sketch of log J).

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_*.py`` (known-answer RNG vectors, closed forms, quadrature
and polynomial exactness, Hutch++ exactness, brute force on tiny inputs, scale
identities).  No function is "parity unpinned".
"""
from .philox import (philox4x64_10, philox4x64_10_np, rademacher, gaussian, probes,
                     PROBE_RADEMACHER, PROBE_GAUSSIAN)
from .spectral import (GERSH_FLOOR_REL, gershgorin_bounds, spectral_interval,
                       oslq_scaling, osa_iop_shift)
from .krylov import windowed_arnoldi
from .quadrature import gauss_quadrature_log, tridiag_from_hessenberg, log_hessenberg_e1
from .estimators import oslq, osa_iop, slq, so_slq, OracleResult, dense_logdet, NotSPDError

__all__ = [
    "philox4x64_10", "philox4x64_10_np", "rademacher", "gaussian", "probes",
    "PROBE_RADEMACHER", "PROBE_GAUSSIAN", "GERSH_FLOOR_REL",
    "gershgorin_bounds", "spectral_interval", "oslq_scaling", "osa_iop_shift",
    "windowed_arnoldi", "gauss_quadrature_log", "tridiag_from_hessenberg",
    "log_hessenberg_e1", "oslq", "osa_iop", "slq", "so_slq", "OracleResult",
    "dense_logdet", "NotSPDError",
]
