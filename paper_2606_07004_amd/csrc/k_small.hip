// OSA-IOP pieces (Alg 2 with Alg 1): log(H_m) e1 per run, the sketch image
// Y = L_c S assembled from the stored Krylov basis, and the per-run
// quadratic forms x^T L_c x / ||x||^2 = sum_t g_t l_t + log(gamma) - c with
// g_t = v_1^T v_t and l = log(H_m) e1.
#include "ld_kernels.h"
#include <algorithm>
#include <cstdint>
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
  if (p >= B || (need && need[p] != 1)) return;
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
  if (p >= B || threadIdx.x != 0 || need_iss[p] != 2) return;
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

// log(H) e1 for a symmetric H, one wave per run: the same symmetry test and
// symmetric tridiagonal part T as k_hess_log_sym, then
//   log(T) e1 = integral over s > 0 of e1/(1+s) - (T + sI)^{-1} e1 ds
// (the Stieltjes form of the logarithm) by the trapezoidal rule in u = log s
// with step 1/2 on [log(a) - 40, log(max(b, 1)) + 40], exact to rounding when
// T's spectrum lies in [a, b].  Each node solves (T + sI) y = e1 by pivots
// eliminated from the bottom (d_t = alpha_t + s, d_i = alpha_i + s -
// e_i^2 / d_{i+1}) and the forward recursion y_1 = 1/d_1,
// y_{i+1} = -e_i y_i / d_{i+1}; component 1 is formed as
// s (d_1 - 1 - s) / ((1+s) d_1) so nothing cancels.  Nodes run on the lanes;
// every component is summed over the lanes by a fixed shuffle tree.
// need[p]: 0 done here, 1 not symmetric (inverse scaling and squaring),
// 2 symmetric but with an eigenvalue outside [a/1000, 1000 b] or longer than
// kTrapMaxDim (QL with logged rotations).
constexpr int kTrapMaxDim = 96;
constexpr double kTrapStep = 0.5;
constexpr double kTrapTail = 40.0;

__device__ inline double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_max64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ inline int sturm_count_below(int nn, const double* al, const double* e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < nn; ++i) {
    q = al[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

__global__ __launch_bounds__(64) void k_hess_log_trap(int B, int m, const double* __restrict__ H,
                                                     const int* __restrict__ meff, double a,
                                                     double b, double symtol, int mode,
                                                     double* __restrict__ ell,
                                                     const double* __restrict__ g, double shift,
                                                     double* __restrict__ K,
                                                     int* __restrict__ flags,
                                                     int* __restrict__ need) {
  __shared__ double al[kTrapMaxDim], ee[kTrapMaxDim], lv[kTrapMaxDim];
  __shared__ double piv[64 * kTrapMaxDim];
  const int p = blockIdx.x, l = threadIdx.x;
  if (p >= B) return;
  const int nn = meff[p];
  if (nn <= 0) {
    if (l == 0) {
      need[p] = 0;
      if (mode == 1) K[p] = 0.0;
    }
    if (mode == 0)
      for (int t = l; t < m; t += 64) ell[(size_t)p * m + t] = 0.0;
    return;
  }
  const double* Hp = H + (size_t)p * (m + 1) * m;
  double hmax = 0.0, asym = 0.0;
  for (int i = l; i < nn; i += 64)
    for (int j = (i > 0 ? i - 1 : 0); j < nn; ++j) {
      const double h = Hp[(size_t)i * m + j];
      hmax = fmax(hmax, fabs(h));
      if (j == i + 1) asym = fmax(asym, fabs(h - Hp[(size_t)j * m + i]));
      else if (j > i + 1) asym = fmax(asym, fabs(h));
    }
  hmax = wave_max64(hmax);
  asym = wave_max64(asym);
  if (!(asym <= symtol * hmax)) {
    if (l == 0) need[p] = 1;
    return;
  }
  if (nn > kTrapMaxDim) {
    if (l == 0) need[p] = 2;
    return;
  }
  for (int i = l; i < nn; i += 64) {
    al[i] = Hp[(size_t)i * m + i];
    ee[i] = (i + 1 < nn) ? 0.5 * (Hp[(size_t)i * m + i + 1] + Hp[(size_t)(i + 1) * m + i]) : 0.0;
    lv[i] = 0.0;
  }
  __syncthreads();
  int outside = 0;
  if (l == 0) outside = sturm_count_below(nn, al, ee, a * 1e-3) > 0;
  if (l == 1) outside = sturm_count_below(nn, al, ee, b * 1e3) < nn;
  outside = __shfl(outside, 0, 64) | __shfl(outside, 1, 64);
  if (outside) {
    if (l == 0) need[p] = 2;
    return;
  }
  const double umin = log(a) - kTrapTail;
  const double umax = log(b > 1.0 ? b : 1.0) + kTrapTail;
  const int nodes = (int)ceil((umax - umin) / kTrapStep) + 1;
  double* dv = piv + (size_t)l * kTrapMaxDim;
  for (int j0 = 0; j0 < nodes; j0 += 64) {
    const int j = j0 + l;
    const bool act = j < nodes;
    const double sv = act ? exp(umin + j * kTrapStep) : 1.0;
    // pivots from the bottom
    double d = al[nn - 1] + sv;
    dv[nn - 1] = d;
    for (int i = nn - 2; i >= 0; --i) {
      d = al[i] + sv - ee[i] * ee[i] / d;
      dv[i] = d;
    }
    // component 1: s (1/(1+s) - 1/d_1) without cancellation
    const double num = (al[0] - 1.0) - (nn >= 2 ? ee[0] * ee[0] / dv[1] : 0.0);
    double c1 = act ? sv * num / ((1.0 + sv) * dv[0]) : 0.0;
    c1 = wave_sum64(c1);
    if (l == 0) lv[0] += c1;
    double y = 1.0 / dv[0];
    for (int i = 1; i < nn; ++i) {
      y = -ee[i - 1] * y / dv[i];
      double ci = act ? -sv * y : 0.0;
      ci = wave_sum64(ci);
      if (l == 0) lv[i] += ci;
    }
  }
  __syncthreads();
  if (l == 0) need[p] = 0;
  if (mode == 0) {
    bool finite = true;
    for (int t = l; t < m; t += 64) {
      const double v = (t < nn) ? lv[t] * kTrapStep : 0.0;
      finite = finite && isfinite(v);
      ell[(size_t)p * m + t] = v;
    }
    if (!finite) flags[p] |= 1;
  } else {
    double acc = 0.0;
    for (int t = l; t < nn; t += 64) acc = fma(g[(size_t)p * (m + 1) + t], lv[t] * kTrapStep, acc);
    acc = wave_sum64(acc) + shift;
    if (l == 0) {
      if (!isfinite(acc)) flags[p] |= 1;
      K[p] = acc;
    }
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
                                                     double* __restrict__ Y, int ldy,
                                                     int accumulate) {
  const int64_t total = n * ld;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kThreads) {
    const int col = (int)(e % ld);
    const int64_t row = e / ld;
    double acc = accumulate ? Y[row * ldy + col] : 0.0;
    for (int t = 0; t < nt; ++t)
      acc = fma(coef[(size_t)t * ld + col], double(slots[(size_t)t * slot_elems + e]), acc);
    Y[row * ldy + col] = acc;
  }
}

// The same sums, 16 bytes of a row per thread (one coalesced stream per basis
// block, four blocks' loads in flight) with the coefficients in LDS; each
// element keeps the FMA chain over t in ascending order, so the result is
// bitwise that of k_combine.
template <typename XT>
__global__ __launch_bounds__(kThreads) void k_combine16(int64_t n, int ld, int nt,
                                                       const XT* __restrict__ slots,
                                                       size_t slot_elems,
                                                       const double* __restrict__ coef,
                                                       double* __restrict__ Y, int accumulate) {
  constexpr int VEC = 16 / sizeof(XT);
  typedef XT xv __attribute__((ext_vector_type(VEC)));
  extern __shared__ double cs[];  // [nt][ld]
  for (int i = threadIdx.x; i < nt * ld; i += kThreads) cs[i] = coef[i];
  __syncthreads();
  const int nch = ld / VEC;
  const int64_t total = n * nch;
  for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kThreads) {
    const int64_t row = q / nch;
    const int col = (int)(q - row * nch) * VEC;
    const size_t off = (size_t)row * ld + col;
    // the FMA chain continues from the stored partial sum when accumulating
    // (the same sequence as one pass over every term)
    double acc[VEC];
    if (accumulate) {
#pragma unroll
      for (int e = 0; e < VEC; e += 2) {
        const double2 y = *reinterpret_cast<const double2*>(Y + off + e);
        acc[e] = y.x;
        acc[e + 1] = y.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = 0.0;
    }
    int t = 0;
    for (; t + 4 <= nt; t += 4) {
      xv x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        x[u] = __builtin_nontemporal_load(
            reinterpret_cast<const xv*>(slots + (size_t)(t + u) * slot_elems + off));
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          acc[e] = fma(cs[(t + u) * ld + col + e], double(x[u][e]), acc[e]);
    }
    for (; t < nt; ++t) {
      const xv x = __builtin_nontemporal_load(
          reinterpret_cast<const xv*>(slots + (size_t)t * slot_elems + off));
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = fma(cs[t * ld + col + e], double(x[e]), acc[e]);
    }
#pragma unroll
    for (int e = 0; e < VEC; e += 2) {
      double2 o;
      o.x = acc[e];
      o.y = acc[e + 1];
      *reinterpret_cast<double2*>(Y + off + e) = o;
    }
  }
}

// Up to kMaxFill ranges of 32-bit words, grid-stride over the concatenation.
struct FillArgs {
  FillItem it[kMaxFill];
  size_t end[kMaxFill];  // running sums of n32
  int count;
};
__global__ __launch_bounds__(kThreads) void k_fill(FillArgs a) {
  const size_t total = a.end[a.count - 1];
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (size_t)gridDim.x * kThreads) {
    int r = 0;
    while (i >= a.end[r]) ++r;
    const size_t j = i - (r ? a.end[r - 1] : 0);
    static_cast<uint32_t*>(a.it[r].p)[j] = a.it[r].val;
  }
}

hipError_t launch_fill(hipStream_t st, const FillItem* items, int count) {
  if (count < 1 || count > kMaxFill || !items) return hipErrorInvalidValue;
  FillArgs a{};
  size_t run = 0;
  for (int r = 0; r < count; ++r) {
    if (!items[r].p && items[r].n32) return hipErrorInvalidValue;
    a.it[r] = items[r];
    run += items[r].n32;
    a.end[r] = run;
  }
  a.count = count;
  if (run == 0) return hipSuccess;
  const size_t nb = std::min<size_t>((run + kThreads - 1) / kThreads, 4 * kMaxBlocks);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_copy_words(uint32_t* __restrict__ dst,
                                                        const uint32_t* __restrict__ src,
                                                        size_t n32) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n32;
       i += (size_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

hipError_t launch_copy_words(hipStream_t st, void* dst, const void* src, size_t n32) {
  if (n32 == 0) return hipSuccess;
  if (!dst || !src) return hipErrorInvalidValue;
  const size_t nb = std::min<size_t>((n32 + kThreads - 1) / kThreads, kMaxBlocks);
  hipLaunchKernelGGL(k_copy_words, dim3((unsigned)nb), dim3(kThreads), 0, st,
                     static_cast<uint32_t*>(dst), static_cast<const uint32_t*>(src), n32);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_pack_results(int ld, const double* __restrict__ K,
                                                          const double* __restrict__ norm2,
                                                          const int* __restrict__ meff,
                                                          const int* __restrict__ flags,
                                                          const int* __restrict__ dflag,
                                                          const int* __restrict__ meff0,
                                                          char* __restrict__ out) {
  double* oK = reinterpret_cast<double*>(out);
  double* oN = oK + ld;
  int* oM = reinterpret_cast<int*>(oN + ld);
  int* oF = oM + ld;
  int* oD = oF + ld;
  int* oM0 = oD + 4;
  for (int i = threadIdx.x; i < ld; i += kThreads) {
    oK[i] = K[i];
    oN[i] = norm2[i];
    oM[i] = meff[i];
    oF[i] = flags[i];
    oM0[i] = meff0 ? meff0[i] : 0;
  }
  if (threadIdx.x < 4) oD[threadIdx.x] = dflag[threadIdx.x];
}

hipError_t launch_pack_results(hipStream_t st, int ld, const double* K, const double* norm2,
                               const int* meff, const int* flags, const int* dflag,
                               const int* meff0, void* out) {
  if (ld < 1 || !K || !norm2 || !meff || !flags || !dflag || !out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_results, dim3(1), dim3(kThreads), 0, st, ld, K, norm2, meff, flags,
                     dflag, meff0, static_cast<char*>(out));
  return hipGetLastError();
}

// Plain copy, 16 bytes per lane, grid-stride (calibration of byte counters).
__global__ __launch_bounds__(kThreads) void k_copy16(const float4* __restrict__ a,
                                                    float4* __restrict__ b, size_t n16) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += stride) b[i] = a[i];
}

// Streaming probe of attainable bandwidth at a given read:write mix: R
// streams read and (W = 1) one written.  The sweep is the Krylov kernels'
// (one resident wave of blocks, the grid a multiple of 8, each round's
// chunks banded per XCD): a chunk is 1024 16-byte elements, each thread
// taking four of them 256 elements apart, all four loads in flight before
// the stores.  With W = 0 each thread keeps a running sum and stores it once
// (so the reads are not dropped).
template <int R, int W>
__global__ __launch_bounds__(kThreads) void k_stream_rw(const float4* __restrict__ a0,
                                                       const float4* __restrict__ a1,
                                                       const float4* __restrict__ a2,
                                                       float4* __restrict__ out,
                                                       float* __restrict__ sink, size_t n16) {
  // the fastest plain stream measured on this part: four 16-byte items per
  // lane in flight, streaming (non-temporal) loads and stores, many short
  // blocks, consecutive groups of items on consecutive blocks
  constexpr int kPer = 4;
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4* b0 = reinterpret_cast<const f4*>(a0);
  const f4* b1 = reinterpret_cast<const f4*>(a1);
  const f4* b2 = reinterpret_cast<const f4*>(a2);
  f4* o = reinterpret_cast<f4*>(out);
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  const size_t stride = (size_t)gridDim.x * kThreads * kPer;
  for (size_t e0 = (size_t)blockIdx.x * kThreads * kPer + threadIdx.x; e0 < n16; e0 += stride) {
    f4 v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const size_t e = e0 + (size_t)u * kThreads;
      v[u] = f4{0.f, 0.f, 0.f, 0.f};
      if (e < n16) {
        v[u] = __builtin_nontemporal_load(b0 + e);
        if (R > 1) v[u] += __builtin_nontemporal_load(b1 + e);
        if (R > 2) v[u] += __builtin_nontemporal_load(b2 + e);
      }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const size_t e = e0 + (size_t)u * kThreads;
      if (e < n16) {
        if (W) __builtin_nontemporal_store(v[u], o + e); else acc += v[u];
      }
    }
  }
  // read-only streams: the sum is stored only if it is not a number (the
  // inputs are finite), which keeps the loads without a write per thread
  if (!W) {
    const float t = acc.x + acc.y + acc.z + acc.w;
    if (t != t) sink[((size_t)blockIdx.x * kThreads + threadIdx.x) % ((size_t)kMaxBlocks * kThreads)] = t;
  }
}

hipError_t launch_stream_rw(hipStream_t st, int reads, int writes, const void* const* src, void* dst,
                            float* sink, size_t bytes) {
  const size_t n16 = bytes / 16;
  if (!src || n16 == 0 || reads < 1 || reads > 3 || writes < 0 || writes > 1 ||
      (writes && !dst) || (!writes && !sink))
    return hipErrorInvalidValue;
  for (int r = 0; r < reads; ++r)
    if (!src[r]) return hipErrorInvalidValue;
  const float4* a0 = static_cast<const float4*>(src[0]);
  const float4* a1 = reads > 1 ? static_cast<const float4*>(src[1]) : nullptr;
  const float4* a2 = reads > 2 ? static_cast<const float4*>(src[2]) : nullptr;
  float4* o = static_cast<float4*>(dst);
  // up to 32768 blocks of 4 x 256 items each per round
  const size_t groups = (n16 + (size_t)kThreads * 4 - 1) / ((size_t)kThreads * 4);
  const dim3 grid((unsigned)std::min<size_t>(groups, 32768)), block(kThreads);
#define LD_STREAM(RR, WW) \
  hipLaunchKernelGGL((k_stream_rw<RR, WW>), grid, block, 0, st, a0, a1, a2, o, sink, n16)
  if (writes) {
    if (reads == 1) LD_STREAM(1, 1); else if (reads == 2) LD_STREAM(2, 1); else LD_STREAM(3, 1);
  } else {
    if (reads == 1) LD_STREAM(1, 0); else if (reads == 2) LD_STREAM(2, 0); else LD_STREAM(3, 0);
  }
#undef LD_STREAM
  return hipGetLastError();
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
                           double a, double b, double* work, int wstride, int mode, double* ell,
                           const double* g, double shift, double* K, int* flags, double symtol,
                           int* need) {
  if (B < 1 || m < 1 || !H || !meff || !work || wstride < hess_log_wstride(m) || !flags ||
      !need || (mode == 0 && !ell) || (mode == 1 && (!g || !K)) || !(a > 0.0) || !(b >= a))
    return hipErrorInvalidValue;
  static const LogRule rule = make_log_rule();
  // symmetric runs: trapezoidal Stieltjes rule; those it leaves (need = 2):
  // QL with logged rotations; non-symmetric ones (need = 1): inverse scaling
  // and squaring
  hipLaunchKernelGGL(k_hess_log_trap, dim3(B), dim3(64), 0, st, B, m, H, meff, a, b, symtol, mode,
                     ell, g, shift, K, flags, need);
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
                          size_t slot_elems, const double* coef, double* Y, int ldy,
                          bool accumulate) {
  const int acc = accumulate ? 1 : 0;
  if (n < 1 || ld < 1 || nt < 1 || !slots || !coef || !Y || ldy != ld ||
      slot_elems < (size_t)n * ld)
    return hipErrorInvalidValue;
  // vectorised form: whole 16-byte chunks per row, coefficients within 48 KB
  // of LDS, 16-byte aligned blocks
  const int vec = xbytes > 0 ? 16 / xbytes : 0;
  const size_t lds = (size_t)nt * ld * 8;
  if (vec > 0 && ld % vec == 0 && lds <= 48 * 1024 && slot_elems % vec == 0 &&
      reinterpret_cast<uintptr_t>(slots) % 16 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0) {
    const int64_t chunks = n * (ld / vec);
    const int64_t nb = std::min<int64_t>((chunks + kThreads - 1) / kThreads, kMaxBlocks);
    if (xbytes == 8)
      hipLaunchKernelGGL(k_combine16<double>, dim3((unsigned)nb), dim3(kThreads), lds, st, n, ld,
                         nt, static_cast<const double*>(slots), slot_elems, coef, Y, acc);
    else if (xbytes == 4)
      hipLaunchKernelGGL(k_combine16<float>, dim3((unsigned)nb), dim3(kThreads), lds, st, n, ld,
                         nt, static_cast<const float*>(slots), slot_elems, coef, Y, acc);
    else if (xbytes == 2)
      hipLaunchKernelGGL(k_combine16<_Float16>, dim3((unsigned)nb), dim3(kThreads), lds, st, n, ld,
                         nt, static_cast<const _Float16*>(slots), slot_elems, coef, Y, acc);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  const int64_t total = n * ld;
  int64_t nb = (total + kThreads - 1) / kThreads;
  if (nb > 4 * kMaxBlocks) nb = 4 * kMaxBlocks;
  if (xbytes == 8)
    hipLaunchKernelGGL(k_combine<double>, dim3((unsigned)nb), dim3(kThreads), 0, st, n, ld, nt,
                       static_cast<const double*>(slots), slot_elems, coef, Y, ldy, acc);
  else if (xbytes == 4)
    hipLaunchKernelGGL(k_combine<float>, dim3((unsigned)nb), dim3(kThreads), 0, st, n, ld, nt,
                       static_cast<const float*>(slots), slot_elems, coef, Y, ldy, acc);
  else if (xbytes == 2)
    hipLaunchKernelGGL(k_combine<_Float16>, dim3((unsigned)nb), dim3(kThreads), 0, st, n, ld, nt,
                       static_cast<const _Float16*>(slots), slot_elems, coef, Y, ldy, acc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace ld
