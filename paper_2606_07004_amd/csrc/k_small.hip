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
                                                      int* __restrict__ flags,
                                                      const int* __restrict__ need) {
  __shared__ double shd[kThreads + 4];
  __shared__ int shi[kThreads + 4];
  const int p = blockIdx.x;
  if (p >= B || (need && !need[p])) return;
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

// Fast path for log(H) e1.  For an SPD operator the windowed recurrence
// gives an H that is symmetric tridiagonal up to rounding (h_{t-1,t} equals
// h_{t,t-1} and the entries above the first superdiagonal vanish in exact
// arithmetic).  When the measured asymmetry is below symtol * max|h|, H is
// replaced by its symmetric tridiagonal part T and log(T) e1 = U log(Theta)
// U^T e1 is formed from the implicit QL iteration: U^T e1 is its first-row
// output and U y is replayed from the logged rotations - O(m^2) work on one
// lane.  Otherwise need_iss[p] = 1 and the general routine (k_hess_log)
// takes the run.  One wave per run; lane 0 works (the QL sweep counts of
// different runs diverge).
__global__ void k_hess_log_sym(int B, int m, const double* __restrict__ H,
                               const int* __restrict__ meff, double* __restrict__ work,
                               int wstride, double symtol, int mode, double* __restrict__ ell,
                               const double* __restrict__ g, double shift,
                               double* __restrict__ K, int* __restrict__ flags,
                               int* __restrict__ need_iss) {
  const int p = blockIdx.x;
  if (p >= B || threadIdx.x != 0) return;
  const int nn = meff[p];
  need_iss[p] = 0;
  if (nn <= 0) {
    if (mode == 0)
      for (int t = 0; t < m; ++t) ell[(size_t)p * m + t] = 0.0;
    else
      K[p] = 0.0;
    return;
  }
  const double* Hp = H + (size_t)p * (m + 1) * m;
  double hmax = 0.0, asym = 0.0;
  for (int i = 0; i < nn; ++i)
    for (int j = (i > 0 ? i - 1 : 0); j < nn; ++j) {
      const double h = Hp[(size_t)i * m + j];
      hmax = fmax(hmax, fabs(h));
      if (j == i + 1) asym = fmax(asym, fabs(h - Hp[(size_t)j * m + i]));
      else if (j > i + 1) asym = fmax(asym, fabs(h));
    }
  if (!(asym <= symtol * hmax)) {
    need_iss[p] = 1;
    return;
  }
  const int cap = 4 * nn * nn;
  double* ws = work + (size_t)p * wstride;
  double* rc = ws;
  double* rs = ws + cap;
  int* ri = reinterpret_cast<int*>(ws + 2 * cap);
  double* d = ws + 2 * cap + (cap + 1) / 2;
  double* e = d + nn;
  double* z = e + nn;
  for (int i = 0; i < nn; ++i) {
    d[i] = Hp[(size_t)i * m + i];
    e[i] = (i + 1 < nn) ? 0.5 * (Hp[(size_t)i * m + i + 1] + Hp[(size_t)(i + 1) * m + i]) : 0.0;
  }
  int nrot = 0;
  const int st = tridiag_ql_first_row(nn, d, e, z, 1, rc, rs, ri, cap, &nrot);
  if (st != 0 || nrot < 0) {
    need_iss[p] = 1;
    return;
  }
  bool ok = true;
  for (int k = 0; k < nn; ++k) {
    if (!(d[k] > 0.0)) ok = false;
    z[k] = (d[k] > 0.0) ? z[k] * log(d[k]) : 0.0;  // y = log(Theta) U^T e1
  }
  if (!ok) flags[p] |= 2;
  apply_logged_rotations(nrot, rc, rs, ri, z, 1);   // U y = log(T) e1
  if (mode == 0) {
    for (int t = 0; t < m; ++t) ell[(size_t)p * m + t] = (t < nn) ? z[t] : 0.0;
  } else {
    double acc = 0.0;
    for (int t = 0; t < nn; ++t) acc = fma(g[(size_t)p * (m + 1) + t], z[t], acc);
    acc += shift;
    if (!isfinite(acc)) flags[p] |= 1;
    K[p] = acc;
  }
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

// Plain copy, 16 bytes per lane, grid-stride (calibration of byte counters).
__global__ __launch_bounds__(kThreads) void k_copy16(const float4* __restrict__ a,
                                                    float4* __restrict__ b, size_t n16) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += stride) b[i] = a[i];
}

hipError_t launch_copy16(hipStream_t st, const void* src, void* dst, size_t bytes) {
  const size_t n16 = bytes / 16;
  if (!src || !dst || n16 == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy16, dim3(4 * kMaxBlocks), dim3(kThreads), 0, st,
                     static_cast<const float4*>(src), static_cast<float4*>(dst), n16);
  return hipGetLastError();
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

int hess_log_wstride(int m) { return 10 * m * m + 8 * m; }

hipError_t launch_hess_log(hipStream_t st, int B, int m, const double* H, const int* meff,
                           double* work, int wstride, int mode, double* ell, const double* g,
                           double shift, double* K, int* flags, double symtol, int* need) {
  if (B < 1 || m < 1 || !H || !meff || !work || wstride < hess_log_wstride(m) || !flags ||
      !need || (mode == 0 && !ell) || (mode == 1 && (!g || !K)))
    return hipErrorInvalidValue;
  static const LogRule rule = make_log_rule();
  hipLaunchKernelGGL(k_hess_log_sym, dim3(B), dim3(64), 0, st, B, m, H, meff, work, wstride, symtol,
                     mode, ell, g, shift, K, flags, need);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hess_log, dim3(B), dim3(kThreads), 0, st, B, m, H, meff, work, wstride, rule,
                     mode, ell, g, shift, K, flags, (const int*)need);
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
