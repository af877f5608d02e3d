// Host-side launchers of the liblogdet device kernels.  Every launcher checks
// the shapes its kernel and grid assume and returns hipErrorInvalidValue
// instead of launching when they do not hold.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ld_device.h"

namespace ld {

enum ValueType : int { VT_F64 = 0, VT_F32 = 1, VT_BF16 = 2 };

constexpr int kMaxBlocks = 2048;  // 256 CUs x 8 resident 256-thread blocks

// Row partition of an [n][ld] probe block shared by the streaming kernels:
// every block owns rows [b*rpb, min(n, (b+1)*rpb)); a row is handled by G
// lanes, each touching `vec` consecutive columns (16 bytes) per access.
// The partition fixes the order of every reduction, so results are bitwise
// reproducible for a given (n, ld, element size).
struct Geom {
  int64_t n = 0;
  int ld = 0;      // leading dimension (multiple of 4)
  int xbytes = 8;  // element size: 8 (FP64) or 4 (FP32)
  int vec = 2;
  int ncolv = 0;   // ld / vec
  int G = 1;       // lanes per row (power of two, <= 64)
  int nblk = 0;
  int rpb = 0;     // rows per block
};
Geom make_geom(int64_t n, int ld, int xbytes);

// Columns col0 .. col0+ncols-1 of X: probe columns pbase .. pbase+nvalid-1,
// then zeros up to ncols (padding).
hipError_t launch_rademacher(hipStream_t st, uint64_t seed, int64_t n, int pbase, int ncols,
                             int nvalid, void* X, int xbytes, int ld, int col0);

// W = opscale * diag(xmult) applied per column to (Q X); X, W share ld/type.
hipError_t launch_spmm(hipStream_t st, const Geom& g, const int* rp, const int* ci,
                       const void* va, int vt, const void* X, void* W,
                       const double* xmult, double opscale);

// part[b][voff+v][col] = mult_v[col] * sum_{rows of b} x_v[row][col] * w[row][col]
hipError_t launch_dots(hipStream_t st, const Geom& g, const void* W, const VecSet& vs, int nv,
                       int voff, int nvtot, double* part);

// w[row][col] -= sum_v d[voff+v][col] * mult_v[col] * x_v[row][col]; when
// want_norm: part[b][0][col] = sum w^2, part[b][1][col] = v1mult[col] *
// sum v1[row][col] w[row][col] (zero when v1 is null).
hipError_t launch_update(hipStream_t st, const Geom& g, void* W, const VecSet& vs, int nv,
                         const double* d, int voff, int want_norm, const void* v1,
                         const double* v1mult, double* part);

// out[i] = sum_{b < nblk} part[b*width + i], fixed order.
hipError_t launch_reduce(hipStream_t st, const double* part, int nblk, int width, double* out);

// Per-probe bookkeeping (B real probes, ld columns).
hipError_t launch_start_finish(hipStream_t st, int B, int ld, const double* nsum, double* norm2,
                               double* mult0, int* active, int* meff, double* g, int gstride);
hipError_t launch_step_finish(hipStream_t st, int B, int ld, int t, int m, const double* d, int j0,
                              int nv, const double* ns, double tol, double* H, int* meff,
                              int* active, double* mult_next, double* g, int* flags);

// Gauss quadrature of log on each probe's T (diag h_tt, subdiag h_t+1,t).
hipError_t launch_gauss_log(hipStream_t st, int B, int m, const double* H, const int* meff,
                            double* work, double* K, int* flags);

// Dense pieces of the Hutch++ sketch (FP64).
// part[b][i][j] = sum_{rows of b} Xa[row][i] * Xb[row][j], i < ca, j < cb
hipError_t launch_gemm_tn(hipStream_t st, const Geom& g, const double* Xa, int lda, int ca,
                          const double* Xb, int ldb, int cb, double* part);
hipError_t launch_chol_inv(hipStream_t st, int s, const double* G, double* work, double* Rinv,
                           int* flag);
hipError_t launch_trsm_rows(hipStream_t st, int64_t n, double* Y, int ld, int s, const double* Rinv);
// X0[row][i] = A[row][i] (i < s); X0[row][s+j] = G[row][j] - sum_i A[row][i] P[i][j];
// part[b][col] = sum over rows of b of X0[row][col]^2 (FP64 values).
hipError_t launch_project(hipStream_t st, const Geom& g, const double* A, int lda, int s,
                          const double* Gm, int ldg, int r, const double* P, void* X0,
                          double* part);

// Matrix set-up.
hipError_t launch_gershgorin(hipStream_t st, int64_t n, const int* rp, const int* ci,
                             const double* va, double* part, int* nparts);

}  // namespace ld
