// OSA-IOP pieces (Alg 2 with Alg 1): log(H_m) e1 per run, the sketch image
// Y = L_c S assembled from the stored Krylov basis, and the per-run
// quadratic forms x^T L_c x / ||x||^2 = sum_t g_t l_t + log(gamma) - c with
// g_t = v_1^T v_t and l = log(H_m) e1.
#include "ld_kernels.h"
#include "gw_ql.h"
#include "hess_log.h"

namespace ld {

// One 256-thread block per run.  mode 0: ell[p][t] = (log H_p e1)_t for
// t < meff (zero beyond).  mode 1: K[p] = sum_t g[p][t] ell_t + shift.
// flags: bit 0 numeric (singular system, square roots not converging, NaN).
__global__ __launch_bounds__(kThreads) void k_hess_log(int B, int m, const double* __restrict__ H,
                                                      const int* __restrict__ meff,
                                                      double* __restrict__ work, int wstride,
                                                      LogRule rule, int mode,
                                                      double* __restrict__ ell,
                                                      const double* __restrict__ g, double shift,
                                                      double* __restrict__ K,
                                                      int* __restrict__ flags) {
  __shared__ double shd[kThreads + 4];
  __shared__ int shi[kThreads + 4];
  const int p = blockIdx.x;
  if (p >= B) return;
  const int nn = meff[p];
  double* ws = work + (size_t)p * wstride;
  double* lv = ws + hess_log_workspace(m);  // [m] result
  if (nn <= 0) {
    if (threadIdx.x == 0) {
      if (mode == 0)
        for (int t = 0; t < m; ++t) ell[(size_t)p * m + t] = 0.0;
      else
        K[p] = 0.0;
    }
    return;
  }
  BlockTeam tm;
  TeamScratch sc{shd, shi};
  const double* Hp = H + (size_t)p * (m + 1) * m;
  const int rc = team_hess_log_e1(tm, nn, Hp, m, lv, ws, sc, rule.x, rule.w);
  if (threadIdx.x != 0) return;
  bool finite = rc == 0;
  if (mode == 0) {
    for (int t = 0; t < m; ++t) {
      const double v = (t < nn && rc == 0) ? lv[t] : 0.0;
      finite = finite && isfinite(v);
      ell[(size_t)p * m + t] = v;
    }
  } else {
    double acc = 0.0;
    for (int t = 0; t < nn; ++t) acc = fma(g[(size_t)p * (m + 1) + t], lv[t], acc);
    acc += shift;
    finite = finite && isfinite(acc);
    K[p] = acc;
  }
  if (!finite) flags[p] |= 1;
}

// coef[t][p] = ||s_p|| ell[p][t] mult_t[p] (t < meff_p) plus (log gamma - c)
// at t = 0: then y_p = sum_t coef[t][p] X_t[:, p] = ||s|| V log(H) e1 +
// (log gamma - c) s, with X_0 = S unnormalised and v_t = mult_t X_t.
__global__ void k_osa_coef(int B, int ld, int m, const double* __restrict__ ell,
                           const double* __restrict__ mult, const double* __restrict__ norm2,
                           const int* __restrict__ meff, double shift, double* __restrict__ coef) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (m + 1) * ld) return;
  const int t = e / ld, p = e % ld;
  double c = 0.0;
  if (p < B) {
    if (t < meff[p]) c = sqrt(norm2[p]) * ell[(size_t)p * m + t] * mult[(size_t)t * ld + p];
    if (t == 0) c += shift;
  }
  coef[e] = c;
}

// Y[row][col] = sum_{t < nt} coef[t][col] X_t[row][col]; X_t = slots + t*slot_elems.
template <typename XT>
__global__ __launch_bounds__(kThreads) void k_combine(int64_t n, int ld, int nt,
                                                     const XT* __restrict__ slots,
                                                     size_t slot_elems,
                                                     const double* __restrict__ coef,
                                                     double* __restrict__ Y, int ldy) {
  const int64_t total = n * ld;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kThreads) {
    const int col = (int)(e % ld);
    const int64_t row = e / ld;
    double acc = 0.0;
    for (int t = 0; t < nt; ++t)
      acc = fma(coef[(size_t)t * ld + col], double(slots[(size_t)t * slot_elems + e]), acc);
    Y[row * ldy + col] = acc;
  }
}

LogRule make_log_rule() {
  LogRule r{};
  double d[kLogNodes], e[kLogNodes], z[kLogNodes];
  for (int j = 0; j < kLogNodes; ++j) {
    d[j] = 0.0;
    e[j] = (j + 1 < kLogNodes) ? (j + 1) / sqrt(4.0 * (j + 1) * (j + 1) - 1.0) : 0.0;
  }
  tridiag_ql_first_row(kLogNodes, d, e, z, 1);
  for (int j = 0; j < kLogNodes; ++j) {
    r.x[j] = 0.5 * (d[j] + 1.0);  // Gauss-Legendre on [0, 1]
    r.w[j] = z[j] * z[j];
  }
  return r;
}

hipError_t launch_hess_log(hipStream_t st, int B, int m, const double* H, const int* meff,
                           double* work, int wstride, int mode, double* ell, const double* g,
                           double shift, double* K, int* flags) {
  if (B < 1 || m < 1 || !H || !meff || !work || wstride < hess_log_workspace(m) + m || !flags ||
      (mode == 0 && !ell) || (mode == 1 && (!g || !K)))
    return hipErrorInvalidValue;
  static const LogRule rule = make_log_rule();
  hipLaunchKernelGGL(k_hess_log, dim3(B), dim3(kThreads), 0, st, B, m, H, meff, work, wstride, rule,
                     mode, ell, g, shift, K, flags);
  return hipGetLastError();
}

hipError_t launch_osa_coef(hipStream_t st, int B, int ld, int m, const double* ell,
                           const double* mult, const double* norm2, const int* meff, double shift,
                           double* coef) {
  if (B < 1 || ld < B || m < 1) return hipErrorInvalidValue;
  const int total = (m + 1) * ld;
  hipLaunchKernelGGL(k_osa_coef, dim3((total + 255) / 256), dim3(256), 0, st, B, ld, m, ell, mult,
                     norm2, meff, shift, coef);
  return hipGetLastError();
}

hipError_t launch_combine(hipStream_t st, int64_t n, int ld, int nt, const void* slots, int xbytes,
                          size_t slot_elems, const double* coef, double* Y, int ldy) {
  if (n < 1 || ld < 1 || nt < 1 || !slots || !coef || !Y || ldy != ld ||
      slot_elems < (size_t)n * ld)
    return hipErrorInvalidValue;
  const int64_t total = n * ld;
  int64_t nb = (total + kThreads - 1) / kThreads;
  if (nb > 4 * kMaxBlocks) nb = 4 * kMaxBlocks;
  if (xbytes == 8)
    hipLaunchKernelGGL(k_combine<double>, dim3((unsigned)nb), dim3(kThreads), 0, st, n, ld, nt,
                       static_cast<const double*>(slots), slot_elems, coef, Y, ldy);
  else
    hipLaunchKernelGGL(k_combine<float>, dim3((unsigned)nb), dim3(kThreads), 0, st, n, ld, nt,
                       static_cast<const float*>(slots), slot_elems, coef, Y, ldy);
  return hipGetLastError();
}

}  // namespace ld
