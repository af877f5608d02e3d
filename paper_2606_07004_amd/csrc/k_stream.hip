// Streaming kernels of the Krylov hot loop: probe generation, the CSR
// product over a probe block, the window inner products, the update/norm
// pass, fixed-order reductions and the per-probe step bookkeeping.
//
// Layout: a probe block is row-major [n][ld] (ld a multiple of 4, padding
// columns held at zero), so one sparse entry gathers one contiguous run of
// probe values.  Every reduction goes through per-block partial sums in a
// fixed order (no floating-point atomics): results are bitwise reproducible.
#include "ld_kernels.h"
#include "gw_ql.h"

namespace ld {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and Rademacher probes.
// Probe column p, row i: block at counter (i / 256, p, 0, 0), key (seed, 0);
// bit i % 64 of word (i / 64) % 4; set -> -1, clear -> +1.
// ---------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3,
                                     uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) { k0 += kW0; k1 += kW1; }
    const uint64_t lo0 = kM0 * c0, hi0 = __umul64hi(kM0, c0);
    const uint64_t lo1 = kM1 * c2, hi1 = __umul64hi(kM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_rademacher(uint64_t seed, int64_t n, int pbase,
                                                        int ncols, int nvalid, T* __restrict__ X,
                                                        int ld, int col0) {
  __shared__ uint64_t words[64][4];
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int cbase = blockIdx.y * 64;
  const int nc = min(64, ncols - cbase);
  if ((int)threadIdx.x < nc) {
    uint64_t c0 = (uint64_t)blockIdx.x, c1 = (uint64_t)(pbase + cbase + (int)threadIdx.x), c2 = 0,
             c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, 0ull);
    words[threadIdx.x][0] = c0;
    words[threadIdx.x][1] = c1;
    words[threadIdx.x][2] = c2;
    words[threadIdx.x][3] = c3;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 256 * nc; e += kThreads) {
    const int rr = e / nc, j = e - (e / nc) * nc;
    const int64_t row = r0 + rr;
    if (row >= n) break;
    const uint64_t w = words[j][(rr >> 6) & 3];
    const T val = ((w >> (rr & 63)) & 1ull) ? T(-1) : T(1);
    X[(size_t)row * ld + col0 + cbase + j] = (cbase + j < nvalid) ? val : T(0);
  }
}

// ---------------------------------------------------------------------------
// CSR x probe block.  G lanes share a row; each lane owns 16 bytes of the
// row's probe vector.  Column index and value are read once per entry by the
// row's lanes (same address, one transaction); the gathered X row segments
// are contiguous.  W = opscale * (Q X) * diag(xmult).
// ---------------------------------------------------------------------------
template <typename VT, typename XT, int G>
__global__ __launch_bounds__(kThreads) void k_spmm(int64_t n, int rpb, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const VT* __restrict__ va,
                                                  const XT* __restrict__ X, XT* __restrict__ W,
                                                  int ld, int ncolv,
                                                  const double* __restrict__ xmult,
                                                  double opscale) {
  using A = typename Acc<XT>::type;
  constexpr int VEC = V16<XT>::N;
  constexpr int RPI = kThreads / G;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t r0 = (int64_t)lb * rpb;
  const int64_t r1 = min(n, r0 + (int64_t)rpb);
  const int rg = threadIdx.x / G, gl = threadIdx.x % G;
  for (int cv = gl; cv < ncolv; cv += G) {
    const int col = cv * VEC;
    double sc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) sc[e] = opscale * (xmult ? xmult[col + e] : 1.0);
    for (int64_t row = r0 + rg; row < r1; row += RPI) {
      A acc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = A(0);
      int k = rp[row];
      const int kend = rp[row + 1];
      for (; k + 4 <= kend; k += 4) {
        int c[4];
        A a[4];
        V16<XT> x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c[u] = ci[k + u];
          a[u] = value_as<VT, A>(va[k + u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u].load(X + (size_t)c[u] * ld + col);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[e] = fma(a[u], x[u].v[e], acc[e]);
      }
      for (; k < kend; ++k) {
        const A a = value_as<VT, A>(va[k]);
        V16<XT> x;
        x.load(X + (size_t)ci[k] * ld + col);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = fma(a, x.v[e], acc[e]);
      }
      V16<XT> out;
#pragma unroll
      for (int e = 0; e < VEC; ++e) out.v[e] = XT(double(acc[e]) * sc[e]);
      out.store(W + (size_t)row * ld + col);
    }
  }
}

// ---------------------------------------------------------------------------
// Window inner products: per block partials of x_v^T w, FP64 accumulation.
// ---------------------------------------------------------------------------
template <typename XT, int G>
__global__ __launch_bounds__(kThreads) void k_dots(int64_t n, int rpb, const XT* __restrict__ W,
                                                  int ld, int ncolv, VecSet vs, int nv, int voff,
                                                  int nvtot, double* __restrict__ part) {
  constexpr int VEC = V16<XT>::N;
  constexpr int RPI = kThreads / G;
  constexpr int CW = G * VEC;
  __shared__ double red[kThreads * VEC];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t r0 = (int64_t)lb * rpb;
  const int64_t r1 = min(n, r0 + (int64_t)rpb);
  const int rg = threadIdx.x / G, gl = threadIdx.x % G;
  const int npass = (ncolv + G - 1) / G;
  for (int pass = 0; pass < npass; ++pass) {
    const int cv = pass * G + gl;
    const bool ok = cv < ncolv;
    const int col = cv * VEC;
    double acc[kMaxNv][VEC];
#pragma unroll
    for (int v = 0; v < kMaxNv; ++v)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[v][e] = 0.0;
    if (ok) {
      for (int64_t row = r0 + rg; row < r1; row += RPI) {
        V16<XT> w;
        w.load(W + (size_t)row * ld + col);
#pragma unroll
        for (int v = 0; v < kMaxNv; ++v) {
          if (v < nv) {
            V16<XT> x;
            x.load(static_cast<const XT*>(vs.x[v]) + (size_t)row * ld + col);
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[v][e] = fma(double(x.v[e]), double(w.v[e]), acc[v][e]);
          }
        }
      }
    }
#pragma unroll
    for (int v = 0; v < kMaxNv; ++v) {
      if (v < nv) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) red[rg * CW + gl * VEC + e] = acc[v][e];
        __syncthreads();
        for (int c = threadIdx.x; c < CW; c += kThreads) {
          double s = 0.0;
          for (int q = 0; q < RPI; ++q) s += red[q * CW + c];
          const int gc = pass * CW + c;
          if (gc < ld) {
            const double m = vs.mult[v] ? vs.mult[v][gc] : 1.0;
            part[((size_t)lb * nvtot + voff + v) * ld + gc] = s * m;
          }
        }
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Orthogonalisation update and the new norm: w -= sum_v h_v v_v.
// ---------------------------------------------------------------------------
template <typename XT, int G>
__global__ __launch_bounds__(kThreads) void k_update(int64_t n, int rpb, XT* __restrict__ W, int ld,
                                                    int ncolv, VecSet vs, int nv,
                                                    const double* __restrict__ d, int voff,
                                                    int want_norm, const XT* __restrict__ v1,
                                                    const double* __restrict__ v1mult,
                                                    double* __restrict__ part) {
  constexpr int VEC = V16<XT>::N;
  constexpr int RPI = kThreads / G;
  constexpr int CW = G * VEC;
  __shared__ double red[2][kThreads * VEC];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t r0 = (int64_t)lb * rpb;
  const int64_t r1 = min(n, r0 + (int64_t)rpb);
  const int rg = threadIdx.x / G, gl = threadIdx.x % G;
  const int npass = (ncolv + G - 1) / G;
  for (int pass = 0; pass < npass; ++pass) {
    const int cv = pass * G + gl;
    const bool ok = cv < ncolv;
    const int col = cv * VEC;
    double coef[kMaxNv][VEC];
    double g1[VEC];
#pragma unroll
    for (int v = 0; v < kMaxNv; ++v)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        coef[v][e] = (ok && v < nv)
                         ? d[(size_t)(voff + v) * ld + col + e] * (vs.mult[v] ? vs.mult[v][col + e] : 1.0)
                         : 0.0;
#pragma unroll
    for (int e = 0; e < VEC; ++e) g1[e] = (ok && v1) ? v1mult[col + e] : 0.0;
    double nacc[VEC], gacc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) { nacc[e] = 0.0; gacc[e] = 0.0; }
    if (ok) {
      for (int64_t row = r0 + rg; row < r1; row += RPI) {
        V16<XT> w;
        w.load(W + (size_t)row * ld + col);
        double wd[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) wd[e] = double(w.v[e]);
#pragma unroll
        for (int v = 0; v < kMaxNv; ++v) {
          if (v < nv) {
            V16<XT> x;
            x.load(static_cast<const XT*>(vs.x[v]) + (size_t)row * ld + col);
#pragma unroll
            for (int e = 0; e < VEC; ++e) wd[e] = fma(-coef[v][e], double(x.v[e]), wd[e]);
          }
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) w.v[e] = XT(wd[e]);
        w.store(W + (size_t)row * ld + col);
        if (want_norm) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) nacc[e] = fma(double(w.v[e]), double(w.v[e]), nacc[e]);
          if (v1) {
            V16<XT> x1;
            x1.load(v1 + (size_t)row * ld + col);
#pragma unroll
            for (int e = 0; e < VEC; ++e) gacc[e] = fma(double(x1.v[e]), double(w.v[e]), gacc[e]);
          }
        }
      }
    }
    if (want_norm) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        red[0][rg * CW + gl * VEC + e] = nacc[e];
        red[1][rg * CW + gl * VEC + e] = gacc[e];
      }
      __syncthreads();
      for (int c = threadIdx.x; c < CW; c += kThreads) {
        double s0 = 0.0, s1 = 0.0;
        for (int q = 0; q < RPI; ++q) {
          s0 += red[0][q * CW + c];
          s1 += red[1][q * CW + c];
        }
        const int gc = pass * CW + c;
        if (gc < ld) {
          part[((size_t)lb * 2 + 0) * ld + gc] = s0;
          part[((size_t)lb * 2 + 1) * ld + gc] = v1 ? s1 * v1mult[gc] : 0.0;
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// out[i] = sum_b part[b][i]: four waves take every fourth block, then the
// four sums are added in a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_reduce(const double* __restrict__ part, int nblk,
                                                    int width, double* __restrict__ out) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (i < width)
    for (int b = w; b < nblk; b += 4) s += part[(size_t)b * width + i];
  sh[w][lane] = s;
  __syncthreads();
  if (w == 0 && i < width) out[i] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

// ---------------------------------------------------------------------------
// Per-probe bookkeeping.
// flags: bit 0 numeric (NaN/Inf), bit 1 non-positive Ritz value / log,
//        bit 2 breakdown (h < tol), bit 3 eigen-iteration did not converge.
// ---------------------------------------------------------------------------
__global__ void k_start_finish(int B, int ld, const double* __restrict__ nsum,
                               double* __restrict__ norm2, double* __restrict__ mult0,
                               int* __restrict__ active, int* __restrict__ meff,
                               double* __restrict__ g, int gstride) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ld) return;
  const double s = (p < B) ? nsum[p] : 0.0;
  norm2[p] = s;
  meff[p] = 0;
  if (p < B && s > 0.0 && isfinite(s)) {
    mult0[p] = 1.0 / sqrt(s);
    active[p] = 1;
  } else {
    mult0[p] = 0.0;
    active[p] = 0;
  }
  if (g && p < B) g[(size_t)p * gstride] = 1.0;
}

__global__ void k_step_finish(int B, int ld, int t, int m, const double* __restrict__ d, int j0,
                              int nv, const double* __restrict__ ns, double tol,
                              double* __restrict__ H, int* __restrict__ meff,
                              int* __restrict__ active, double* __restrict__ mult_next,
                              double* __restrict__ g, int* __restrict__ flags) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ld) return;
  if (p >= B || !active[p]) {
    mult_next[p] = 0.0;
    return;
  }
  double* Hp = H + (size_t)p * (m + 1) * m;
  bool finite = true;
  for (int v = 0; v < nv; ++v) {
    const double h = d[(size_t)v * ld + p];
    finite = finite && isfinite(h);
    Hp[(size_t)(j0 + v) * m + t] = h;
  }
  const double beta = sqrt(ns[p]);
  Hp[(size_t)(t + 1) * m + t] = beta;
  meff[p] = t + 1;
  if (!finite || !isfinite(beta)) {
    flags[p] |= 1;
    active[p] = 0;
    mult_next[p] = 0.0;
    return;
  }
  if (!(beta >= tol)) {
    flags[p] |= 4;
    active[p] = 0;
    mult_next[p] = 0.0;
    return;
  }
  if (g) g[(size_t)p * (m + 1) + t + 1] = ns[ld + p] / beta;
  mult_next[p] = 1.0 / beta;
}

// ---------------------------------------------------------------------------
// Gauss quadrature of log per probe (Golub-Welsch on T = tridiag(h)).
// One thread per probe; the d/e/z work arrays are [m][B] so that consecutive
// threads touch consecutive addresses.
// ---------------------------------------------------------------------------
__global__ void k_gauss_log(int B, int m, const double* __restrict__ H, const int* __restrict__ meff,
                            double* __restrict__ work, double* __restrict__ K,
                            int* __restrict__ flags) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B) return;
  const int nn = meff[p];
  if (nn <= 0) {
    K[p] = 0.0;
    return;
  }
  double* dd = work + p;
  double* ee = work + (size_t)m * B + p;
  double* zz = work + (size_t)2 * m * B + p;
  const double* Hp = H + (size_t)p * (m + 1) * m;
  for (int i = 0; i < nn; ++i) dd[(size_t)i * B] = Hp[(size_t)i * m + i];
  for (int i = 0; i + 1 < nn; ++i) ee[(size_t)i * B] = Hp[(size_t)(i + 1) * m + i];
  const int rc = tridiag_ql_first_row(nn, dd, ee, zz, B);
  int bad = 0;
  const double s = gauss_log_sum(nn, dd, zz, B, &bad);
  if (rc) flags[p] |= 8;
  if (bad) flags[p] |= 2;
  if (!isfinite(s)) flags[p] |= 1;
  K[p] = s;
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

Geom make_geom(int64_t n, int ld, int xbytes) {
  Geom g;
  g.n = n;
  g.ld = ld;
  g.xbytes = xbytes;
  g.vec = 16 / xbytes;
  g.ncolv = ld / g.vec;
  g.G = pow2_at_least(g.ncolv < 1 ? 1 : g.ncolv);
  if (g.G > 64) g.G = 64;
  const int rpi = kThreads / g.G;
  int64_t nb = (n + rpi - 1) / rpi;
  if (nb > kMaxBlocks) nb = kMaxBlocks;
  if (nb < 1) nb = 1;
  g.nblk = (int)nb;
  g.rpb = (int)((n + nb - 1) / nb);
  return g;
}

static bool geom_ok(const Geom& g) {
  return g.n > 0 && g.ld > 0 && g.ld % 4 == 0 && (g.xbytes == 8 || g.xbytes == 4) &&
         g.vec * g.ncolv == g.ld && g.nblk >= 1 && (int64_t)g.nblk * g.rpb >= g.n;
}

#define LD_DISPATCH_G(G, ...)                                   \
  switch (G) {                                                  \
    case 1: { constexpr int GG = 1; __VA_ARGS__; } break;       \
    case 2: { constexpr int GG = 2; __VA_ARGS__; } break;       \
    case 4: { constexpr int GG = 4; __VA_ARGS__; } break;       \
    case 8: { constexpr int GG = 8; __VA_ARGS__; } break;       \
    case 16: { constexpr int GG = 16; __VA_ARGS__; } break;     \
    case 32: { constexpr int GG = 32; __VA_ARGS__; } break;     \
    default: { constexpr int GG = 64; __VA_ARGS__; } break;     \
  }

hipError_t launch_rademacher(hipStream_t st, uint64_t seed, int64_t n, int pbase, int ncols,
                             int nvalid, void* X, int xbytes, int ld, int col0) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if (!X || col0 < 0 || col0 + ncols > ld || pbase < 0 || nvalid < 0 || nvalid > ncols)
    return hipErrorInvalidValue;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((ncols + 63) / 64));
  if (xbytes == 8)
    hipLaunchKernelGGL(k_rademacher<double>, grid, dim3(kThreads), 0, st, seed, n, pbase, ncols,
                       nvalid, static_cast<double*>(X), ld, col0);
  else if (xbytes == 4)
    hipLaunchKernelGGL(k_rademacher<float>, grid, dim3(kThreads), 0, st, seed, n, pbase, ncols,
                       nvalid, static_cast<float*>(X), ld, col0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename VT, typename XT>
static hipError_t spmm_typed(hipStream_t st, const Geom& g, const int* rp, const int* ci,
                             const VT* va, const XT* X, XT* W, const double* xmult, double opscale) {
  LD_DISPATCH_G(g.G, hipLaunchKernelGGL((k_spmm<VT, XT, GG>), dim3(g.nblk), dim3(kThreads), 0, st,
                                        g.n, g.rpb, rp, ci, va, X, W, g.ld, g.ncolv, xmult,
                                        opscale));
  return hipGetLastError();
}

hipError_t launch_spmm(hipStream_t st, const Geom& g, const int* rp, const int* ci, const void* va,
                       int vt, const void* X, void* W, const double* xmult, double opscale) {
  if (!geom_ok(g) || !rp || !ci || !va || !X || !W || X == W) return hipErrorInvalidValue;
  if (g.xbytes == 8) {
    if (vt == VT_F64)
      return spmm_typed<double, double>(st, g, rp, ci, static_cast<const double*>(va),
                                        static_cast<const double*>(X), static_cast<double*>(W),
                                        xmult, opscale);
    if (vt == VT_F32)
      return spmm_typed<float, double>(st, g, rp, ci, static_cast<const float*>(va),
                                       static_cast<const double*>(X), static_cast<double*>(W),
                                       xmult, opscale);
    if (vt == VT_BF16)
      return spmm_typed<uint16_t, double>(st, g, rp, ci, static_cast<const uint16_t*>(va),
                                          static_cast<const double*>(X), static_cast<double*>(W),
                                          xmult, opscale);
  } else {
    if (vt == VT_F32)
      return spmm_typed<float, float>(st, g, rp, ci, static_cast<const float*>(va),
                                      static_cast<const float*>(X), static_cast<float*>(W), xmult,
                                      opscale);
    if (vt == VT_BF16)
      return spmm_typed<uint16_t, float>(st, g, rp, ci, static_cast<const uint16_t*>(va),
                                         static_cast<const float*>(X), static_cast<float*>(W),
                                         xmult, opscale);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dots(hipStream_t st, const Geom& g, const void* W, const VecSet& vs, int nv,
                       int voff, int nvtot, double* part) {
  if (!geom_ok(g) || !W || !part || nv < 1 || nv > kMaxNv || voff < 0 || voff + nv > nvtot)
    return hipErrorInvalidValue;
  for (int v = 0; v < nv; ++v)
    if (!vs.x[v]) return hipErrorInvalidValue;
  if (g.xbytes == 8) {
    LD_DISPATCH_G(g.G, hipLaunchKernelGGL((k_dots<double, GG>), dim3(g.nblk), dim3(kThreads), 0, st,
                                          g.n, g.rpb, static_cast<const double*>(W), g.ld, g.ncolv,
                                          vs, nv, voff, nvtot, part));
  } else {
    LD_DISPATCH_G(g.G, hipLaunchKernelGGL((k_dots<float, GG>), dim3(g.nblk), dim3(kThreads), 0, st,
                                          g.n, g.rpb, static_cast<const float*>(W), g.ld, g.ncolv,
                                          vs, nv, voff, nvtot, part));
  }
  return hipGetLastError();
}

hipError_t launch_update(hipStream_t st, const Geom& g, void* W, const VecSet& vs, int nv,
                         const double* d, int voff, int want_norm, const void* v1,
                         const double* v1mult, double* part) {
  if (!geom_ok(g) || !W || !d || nv < 0 || nv > kMaxNv || (want_norm && !part) ||
      (v1 && !v1mult))
    return hipErrorInvalidValue;
  for (int v = 0; v < nv; ++v)
    if (!vs.x[v]) return hipErrorInvalidValue;
  if (g.xbytes == 8) {
    LD_DISPATCH_G(g.G, hipLaunchKernelGGL((k_update<double, GG>), dim3(g.nblk), dim3(kThreads), 0,
                                          st, g.n, g.rpb, static_cast<double*>(W), g.ld, g.ncolv,
                                          vs, nv, d, voff, want_norm,
                                          static_cast<const double*>(v1), v1mult, part));
  } else {
    LD_DISPATCH_G(g.G, hipLaunchKernelGGL((k_update<float, GG>), dim3(g.nblk), dim3(kThreads), 0,
                                          st, g.n, g.rpb, static_cast<float*>(W), g.ld, g.ncolv, vs,
                                          nv, d, voff, want_norm, static_cast<const float*>(v1),
                                          v1mult, part));
  }
  return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, const double* part, int nblk, int width, double* out) {
  if (!part || !out || nblk < 1 || width < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce, dim3((width + 63) / 64), dim3(kThreads), 0, st, part, nblk, width,
                     out);
  return hipGetLastError();
}

hipError_t launch_start_finish(hipStream_t st, int B, int ld, const double* nsum, double* norm2,
                               double* mult0, int* active, int* meff, double* g, int gstride) {
  if (B < 1 || ld < B) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_start_finish, dim3((ld + 255) / 256), dim3(256), 0, st, B, ld, nsum, norm2,
                     mult0, active, meff, g, gstride);
  return hipGetLastError();
}

hipError_t launch_step_finish(hipStream_t st, int B, int ld, int t, int m, const double* d, int j0,
                              int nv, const double* ns, double tol, double* H, int* meff,
                              int* active, double* mult_next, double* g, int* flags) {
  if (B < 1 || ld < B || t < 0 || t >= m || j0 < 0 || j0 + nv != t + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_step_finish, dim3((ld + 255) / 256), dim3(256), 0, st, B, ld, t, m, d, j0,
                     nv, ns, tol, H, meff, active, mult_next, g, flags);
  return hipGetLastError();
}

hipError_t launch_gauss_log(hipStream_t st, int B, int m, const double* H, const int* meff,
                            double* work, double* K, int* flags) {
  if (B < 1 || m < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gauss_log, dim3((B + 63) / 64), dim3(64), 0, st, B, m, H, meff, work, K,
                     flags);
  return hipGetLastError();
}

}  // namespace ld
