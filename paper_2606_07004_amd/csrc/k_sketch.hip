// Dense pieces of the Hutch++ split (FP64): tall-skinny Gram/cross products,
// the small Cholesky factor and its inverse (CholQR2, the QR of the sketch
// image with a positive diagonal), the row-wise triangular solve, the
// residual projection u = g - A (A^T g), and the matrix set-up kernels.
#include "ld_kernels.h"

namespace ld {

// part[i][j][b] over a 32 x 32 output tile per grid.y; rows staged through
// LDS 64 at a time, each thread accumulating a 2 x 2 micro-tile in row order.
__global__ __launch_bounds__(kThreads) void k_gemm_tn(int64_t n, int rpb, const double* __restrict__ Xa,
                                                     int lda, int ca, const double* __restrict__ Xb,
                                                     int ldb, int cb, double* __restrict__ part) {
  constexpr int TR = 64, TT = 32;
  __shared__ double sa[TR][TT + 1];
  __shared__ double sb[TR][TT + 1];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t r0 = (int64_t)lb * rpb;
  const int64_t r1 = min(n, r0 + (int64_t)rpb);
  const int ntj = (cb + TT - 1) / TT;
  const int ti = blockIdx.y / ntj, tj = blockIdx.y % ntj;
  const int i0 = ti * TT, j0 = tj * TT;
  const int ni = min(TT, ca - i0), nj = min(TT, cb - j0);
  const int t = threadIdx.x;
  const int ii0 = (t >> 4) * 2, jj0 = (t & 15) * 2;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t row0 = r0; row0 < r1; row0 += TR) {
    for (int e = t; e < TR * TT; e += kThreads) {
      const int rr = e / TT, c = e % TT;
      const int64_t row = row0 + rr;
      sa[rr][c] = (row < r1 && c < ni) ? Xa[(size_t)row * lda + i0 + c] : 0.0;
      sb[rr][c] = (row < r1 && c < nj) ? Xb[(size_t)row * ldb + j0 + c] : 0.0;
    }
    __syncthreads();
    const int nr = (int)min((int64_t)TR, r1 - row0);
    for (int rr = 0; rr < nr; ++rr) {
      const double a0 = sa[rr][ii0], a1 = sa[rr][ii0 + 1];
      const double b0 = sb[rr][jj0], b1 = sb[rr][jj0 + 1];
      acc[0][0] = fma(a0, b0, acc[0][0]);
      acc[0][1] = fma(a0, b1, acc[0][1]);
      acc[1][0] = fma(a1, b0, acc[1][0]);
      acc[1][1] = fma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int i = ii0 + x, j = jj0 + y;
      if (i < ni && j < nj) part[((size_t)(i0 + i) * cb + j0 + j) * gridDim.x + lb] = acc[x][y];
    }
}

// Cholesky G = R^T R (R upper, positive diagonal) and R^{-1}, one block.
// flag = 1 when a pivot is not positive or falls below 1e-14 of its column's
// Gram diagonal (the sketch image has numerically lost rank).
// R and Rinv may live in global memory or in LDS (small s): the same
// operations in the same order either way.
// Cholesky factor R of the Gram matrix G = Y^T Y and the inverse of R, with
// columns that are numerically dependent on earlier ones dropped: at step k
// the pivot (in exact arithmetic the squared norm of the part of column k
// orthogonal to the columns kept before it) is compared with the column's
// squared norm G_kk; at or below kRankRtol^2 G_kk (or G_kk = 0) the column
// is dropped: its row of R is zero (so it updates nothing after it) and its
// row and column of the inverse are zero, so Y R^{-1} keeps an orthonormal
// basis of range(Y) in the kept columns, in column order, and zero columns
// in the dropped ones.  A full-rank Y drops nothing.  flag = 1 only for a
// non-finite pivot.
constexpr double kRankRtol = 1e-6;

__device__ inline void chol_inv_body(int s, const double* __restrict__ G, double* __restrict__ R,
                                     double* __restrict__ Rinv, int* __restrict__ flag,
                                     double& piv, int& bad, double* gdiag) {
  const int t = threadIdx.x;
  for (int idx = t; idx < s * s; idx += kThreads) R[idx] = G[idx];
  // the original diagonal (the pivot test) in LDS: no global read per step
  for (int k = t; k < s; k += kThreads) gdiag[k] = G[k * s + k];
  if (t == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < s; ++k) {
    if (t == 0) {
      const double a = R[k * s + k];
      if (!isfinite(a) || !isfinite(gdiag[k])) bad = 1;
      // dropped column: pivot 0 (the test below keeps it out of the inverse)
      piv = (a > kRankRtol * kRankRtol * gdiag[k] && gdiag[k] > 0.0) ? sqrt(a) : 0.0;
      R[k * s + k] = piv;
    }
    __syncthreads();
    if (bad) break;
    if (piv == 0.0) {
      // a dependent column: zero row, nothing to subtract from later columns
      for (int j = k + 1 + t; j < s; j += kThreads) R[k * s + j] = 0.0;
      __syncthreads();
      continue;
    }
    for (int j = k + 1 + t; j < s; j += kThreads) R[k * s + j] /= piv;
    __syncthreads();
    const int rem = s - k - 1;
    for (int idx = t; idx < rem * rem; idx += kThreads) {
      const int i = k + 1 + idx / rem, j = k + 1 + idx % rem;
      if (j >= i) R[i * s + j] -= R[k * s + i] * R[k * s + j];
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) *flag = 1;
    return;
  }
  for (int idx = t; idx < s * s; idx += kThreads)
    if (idx / s > idx % s) R[idx] = 0.0;
  __syncthreads();
  // inverse of the upper triangle by back substitution, one column per
  // thread, over the kept columns (a dropped column j: zero column; a
  // dropped row i: zero entry, so it adds nothing to the rows above)
  for (int j = t; j < s; j += kThreads) {
    for (int i = s - 1; i > j; --i) Rinv[i * s + j] = 0.0;
    if (R[j * s + j] == 0.0) {
      for (int i = j; i >= 0; --i) Rinv[i * s + j] = 0.0;
      continue;
    }
    Rinv[j * s + j] = 1.0 / R[j * s + j];
    for (int i = j - 1; i >= 0; --i) {
      if (R[i * s + i] == 0.0) {
        Rinv[i * s + j] = 0.0;
        continue;
      }
      // sum over l = i+1 .. j in ascending order; four terms' operands
      // loaded before their FMAs
      double acc = 0.0;
      int l = i + 1;
      for (; l + 4 <= j + 1; l += 4) {
        const double r0 = R[i * s + l], r1 = R[i * s + l + 1], r2 = R[i * s + l + 2],
                     r3 = R[i * s + l + 3];
        const double x0 = Rinv[l * s + j], x1 = Rinv[(l + 1) * s + j], x2 = Rinv[(l + 2) * s + j],
                     x3 = Rinv[(l + 3) * s + j];
        acc = fma(r0, x0, acc);
        acc = fma(r1, x1, acc);
        acc = fma(r2, x2, acc);
        acc = fma(r3, x3, acc);
      }
      for (; l <= j; ++l) acc = fma(R[i * s + l], Rinv[l * s + j], acc);
      Rinv[i * s + j] = -acc / R[i * s + i];
    }
  }
  if (t == 0) *flag = 0;
}

__global__ __launch_bounds__(kThreads) void k_chol_inv(int s, const double* __restrict__ G,
                                                      double* __restrict__ R,
                                                      double* __restrict__ Rinv,
                                                      int* __restrict__ flag) {
  __shared__ double piv;
  __shared__ int bad;
  __shared__ double gdiag[256];
  chol_inv_body(s, G, R, Rinv, flag, piv, bad, gdiag);
}

// s <= kCholLdsMax: the factor and its inverse in LDS, copied out at the end
// (each step's barriers then wait on LDS, not on L2 round trips).
constexpr int kCholLdsMax = 64;
__global__ __launch_bounds__(kThreads) void k_chol_inv_lds(int s, const double* __restrict__ G,
                                                          double* __restrict__ R,
                                                          double* __restrict__ Rinv,
                                                          int* __restrict__ flag) {
  extern __shared__ double sm[];
  __shared__ double piv;
  __shared__ int bad;
  double* sR = sm;
  double* sI = sm + (size_t)s * s;
  __shared__ double gdiag[kCholLdsMax];
  chol_inv_body(s, G, sR, sI, flag, piv, bad, gdiag);
  __syncthreads();
  if (bad) return;
  for (int idx = threadIdx.x; idx < s * s; idx += kThreads) {
    R[idx] = sR[idx];
    Rinv[idx] = sI[idx];
  }
}

// Y[row][j] <- sum_i Y[row][i] M[i][j] for j < sout (M is s x sout, row-major;
// with UPPER only i <= j, M upper triangular), 16 rows per block, output
// columns in chunks of 16; the row tile stays in LDS so the update is in place.
template <bool UPPER>
__global__ __launch_bounds__(kThreads) void k_rows_mat(int64_t n, double* __restrict__ Y, int ld,
                                                      int s, const double* __restrict__ M, int sout) {
  extern __shared__ double sm[];
  double* sy = sm;            // [16][s]
  double* sr = sm + 16 * s;   // [s][16]
  const int64_t row0 = (int64_t)blockIdx.x * 16;
  const int t = threadIdx.x;
  const int nr = (int)min((int64_t)16, n - row0);
  for (int e = t; e < 16 * s; e += kThreads) {
    const int rr = e / s, c = e % s;
    sy[e] = (rr < nr) ? Y[(size_t)(row0 + rr) * ld + c] : 0.0;
  }
  for (int j0 = 0; j0 < sout; j0 += 16) {
    const int nc = min(16, sout - j0);
    __syncthreads();
    for (int e = t; e < s * 16; e += kThreads) {
      const int i = e / 16, jj = e % 16;
      sr[e] = (jj < nc) ? M[(size_t)i * sout + j0 + jj] : 0.0;
    }
    __syncthreads();
    const int rr = t / 16, jj = t % 16;
    if (rr < nr && jj < nc) {
      const int j = j0 + jj;
      const int iend = UPPER ? j + 1 : s;
      double acc = 0.0;
      for (int i = 0; i < iend; ++i) acc = fma(sy[rr * s + i], sr[i * 16 + jj], acc);
      Y[(size_t)(row0 + rr) * ld + j] = acc;
    }
  }
}

// Dominant rank-k left singular subspace of Y from its Gram matrix
// G = Y^T Y (q x q): the eigenvectors v_j of G for its k largest eigenvalues
// lambda_j, returned as U[i*k + j] = v_j[i] / sqrt(lambda_j), so that Y U has
// orthonormal columns spanning the k dominant left singular vectors of Y (in
// exact arithmetic; a CholQR pass on Y U removes the rounding).  This needs
// no full-rank factorisation of Y, so a sketch of rank between k and q is
// fine.  Cyclic Jacobi (Golub & Van Loan, the symmetric Schur rotation) with
// the round-robin ordering: in each round the q/2 rotations act on disjoint
// index pairs and are applied together, rows first, then columns and the
// eigenvector matrix V.  Sweeps stop when the off-diagonal mass falls below
// 1e-30 of the diagonal mass (at most 60).  Eigenvalues are taken in
// descending order, ties by index; each v_j has its largest-magnitude
// component (first one on ties) positive.  flag = 1 when the sweeps did not
// converge or lambda_k <= 1e-13 lambda_1 (the sketch has rank below k).
constexpr int kEigMax = kSoSlqMaxSketch;

__global__ __launch_bounds__(kThreads) void k_subspace_eig(int q, int k, const double* __restrict__ G,
                                                          double* __restrict__ U,
                                                          int* __restrict__ flag) {
  __shared__ double M[kEigMax * kEigMax];
  __shared__ double V[kEigMax * kEigMax];
  __shared__ double cs[kEigMax / 2], sn[kEigMax / 2];
  __shared__ int pa[kEigMax / 2], pb[kEigMax / 2];
  __shared__ double red[2][kThreads];
  __shared__ int order[kEigMax];
  const int t = threadIdx.x;
  // symmetrised copy of G (the Gram sums of (i, j) and (j, i) may round apart)
  for (int e = t; e < q * q; e += kThreads) {
    const int i = e / q, j = e % q;
    M[e] = 0.5 * (G[i * q + j] + G[j * q + i]);
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  const int qq = q + (q & 1);       // even number of players; index q is a dummy
  const int np = qq / 2;
  bool converged = q == 1;
  for (int sweep = 0; sweep < 60 && !converged; ++sweep) {
    for (int round = 0; round < qq - 1; ++round) {
      // pairs of the round (circle method: qq-1 players rotate, one is fixed)
      __syncthreads();
      if (t < np) {
        int a, b;
        if (t == 0) {
          a = round;
          b = qq - 1;
        } else {
          a = (round + t) % (qq - 1);
          b = (round - t + (qq - 1)) % (qq - 1);
        }
        const int p = min(a, b), r = max(a, b);
        double c = 1.0, s = 0.0;
        if (r < q) {
          const double app = M[p * q + p], arr = M[r * q + r], apr = M[p * q + r];
          if (apr != 0.0) {
            const double tau = (arr - app) / (2.0 * apr);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        pa[t] = p;
        pb[t] = r;
        cs[t] = c;
        sn[t] = s;
      }
      __syncthreads();
      // rows p, r of every pair: M <- J^T M
      for (int e = t; e < np * q; e += kThreads) {
        const int w = e / q, j = e % q;
        const int p = pa[w], r = pb[w];
        if (r >= q || sn[w] == 0.0) continue;
        const double mp = M[p * q + j], mr = M[r * q + j];
        M[p * q + j] = cs[w] * mp - sn[w] * mr;
        M[r * q + j] = sn[w] * mp + cs[w] * mr;
      }
      __syncthreads();
      // columns p, r: M <- M J, V <- V J
      for (int e = t; e < np * q; e += kThreads) {
        const int w = e / q, i = e % q;
        const int p = pa[w], r = pb[w];
        if (r >= q || sn[w] == 0.0) continue;
        const double mp = M[i * q + p], mr = M[i * q + r];
        M[i * q + p] = cs[w] * mp - sn[w] * mr;
        M[i * q + r] = sn[w] * mp + cs[w] * mr;
        const double vp = V[i * q + p], vr = V[i * q + r];
        V[i * q + p] = cs[w] * vp - sn[w] * vr;
        V[i * q + r] = sn[w] * vp + cs[w] * vr;
      }
    }
    __syncthreads();
    double off = 0.0, dia = 0.0;
    for (int e = t; e < q * q; e += kThreads) {
      const double v = M[e] * M[e];
      if (e / q == e % q) dia += v; else off += v;
    }
    red[0][t] = off;
    red[1][t] = dia;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (t < w) {
        red[0][t] += red[0][t + w];
        red[1][t] += red[1][t + w];
      }
      __syncthreads();
    }
    converged = red[0][0] <= 1e-30 * red[1][0];
    __syncthreads();
  }
  if (t == 0) {
    // k largest eigenvalues, descending, ties by index
    for (int i = 0; i < q; ++i) order[i] = i;
    for (int i = 0; i < k; ++i) {
      int best = i;
      for (int j = i + 1; j < q; ++j) {
        const double vj = M[order[j] * q + order[j]], vb = M[order[best] * q + order[best]];
        if (vj > vb || (vj == vb && order[j] < order[best])) best = j;
      }
      const int tmp = order[i];
      order[i] = order[best];
      order[best] = tmp;
    }
    const double l1 = M[order[0] * q + order[0]], lk = M[order[k - 1] * q + order[k - 1]];
    *flag = (converged && lk > 1e-13 * l1 && lk > 0.0) ? 0 : 1;
  }
  __syncthreads();
  for (int j = t; j < k; j += kThreads) {
    const int col = order[j];
    int imax = 0;
    double vmax = -1.0;
    for (int i = 0; i < q; ++i) {
      const double a = fabs(V[i * q + col]);
      if (a > vmax) {
        vmax = a;
        imax = i;
      }
    }
    const double lam = M[col * q + col];
    const double sc = (V[imax * q + col] >= 0.0 ? 1.0 : -1.0) / sqrt(lam > 0.0 ? lam : 1.0);
    for (int i = 0; i < q; ++i) U[i * k + j] = sc * V[i * q + col];
  }
}

// ---------------------------------------------------------------------------
// FP64 matrix-core (MFMA) versions of the tall-skinny contractions of the
// sketch: Gram blocks X_a^T X_b, rows times a small matrix, and the
// projection of the residual probes.  v_mfma_f64_16x16x4f64 multiplies a
// 16 x 4 block by a 4 x 16 block into a 16 x 16 accumulator; its lanes
// (measured on gfx950): lane l carries A[l % 16][l / 16] and B[l / 16][l % 16],
// and element e of lane l's accumulator is D[4 e + l / 16][l % 16].
// ---------------------------------------------------------------------------
typedef double dmf4 __attribute__((ext_vector_type(4)));

__device__ inline dmf4 mfma_f64(double a, double b, dmf4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// part[i][j][block] = sum over the block's rows of Xa[row][i] Xb[row][j]:
// one block of 4 waves per (row block, group of TI x TJ output tiles of
// 16 x 16); each wave takes a quarter of the block's rows (the k dimension of
// the product is the row index, 4 rows per instruction) and the four waves'
// sums are added in wave order.
template <int TI, int TJ, bool MASK>
__global__ __launch_bounds__(kThreads) void k_gemm_tn_mfma(int64_t n, int rpb, const double* __restrict__ Xa,
                                                          int lda, int ca, const double* __restrict__ Xb,
                                                          int ldb, const uint64_t* __restrict__ Mb,
                                                          int nwb, int cb, int ngj,
                                                          double* __restrict__ part) {
  __shared__ double red[3][TI * TJ * 4][64];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int gi = blockIdx.y / ngj, gj = blockIdx.y % ngj;
  const int b = blockIdx.x;
  const int64_t b0 = (int64_t)b * rpb;
  const int64_t b1 = min(n, b0 + (int64_t)rpb);
  const int64_t q = (((b1 - b0) + 15) / 16) * 4;  // rows per wave, a multiple of 4
  const int64_t r0 = min(b1, b0 + w * q);
  const int64_t r1 = min(b1, r0 + q);
  const int kr = l >> 4, cl = l & 15;
  int ia[TI], jb[TJ];
  bool oka[TI], okb[TJ];
#pragma unroll
  for (int t = 0; t < TI; ++t) {
    ia[t] = (gi * TI + t) * 16 + cl;
    oka[t] = ia[t] < ca;
  }
#pragma unroll
  for (int t = 0; t < TJ; ++t) {
    jb[t] = (gj * TJ + t) * 16 + cl;
    okb[t] = jb[t] < cb;
  }
  dmf4 acc[TI][TJ];
#pragma unroll
  for (int x = 0; x < TI; ++x)
#pragma unroll
    for (int y = 0; y < TJ; ++y) acc[x][y] = dmf4{0.0, 0.0, 0.0, 0.0};
  // a Gram product (the same block on both sides, diagonal tile group):
  // the B operand is the A operand already loaded
  const bool same = TI == TJ && Xa == Xb && lda == ldb && gi == gj && ca == cb;
  // sign words: the TJ tiles of 16 columns from jb[0] lie in one 64-column word
  const int wb = jb[0] >> 6;
  // four groups of 4 rows per round: their loads are issued together, then
  // the products run in row order (the same accumulation order as one group
  // at a time)
  constexpr int U = 4;
  for (int64_t base = r0; base < r1; base += 4 * U) {
    double a[U][TI], bd[U][TJ];
    uint64_t wd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = base + 4 * u + kr;
      const bool okr = row < r1;
#pragma unroll
      for (int t = 0; t < TI; ++t)
        a[u][t] = (okr && oka[t]) ? Xa[(size_t)row * lda + ia[t]] : 0.0;
      if constexpr (MASK) {
        wd[u] = okr ? Mb[(size_t)row * nwb + wb] : 0ull;
      } else {
#pragma unroll
        for (int t = 0; t < TJ; ++t)
          bd[u][t] = (!same && okr && okb[t]) ? Xb[(size_t)row * ldb + jb[t]] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool okr = base + 4 * u + kr < r1;
      double bb[TJ];
#pragma unroll
      for (int t = 0; t < TJ; ++t) {
        if constexpr (MASK)
          bb[t] = (okr && okb[t]) ? (((wd[u] >> (jb[t] & 63)) & 1ull) ? -1.0 : 1.0) : 0.0;
        else
          bb[t] = (same && t < TI) ? a[u][t] : bd[u][t];
      }
#pragma unroll
      for (int x = 0; x < TI; ++x)
#pragma unroll
        for (int y = 0; y < TJ; ++y) acc[x][y] = mfma_f64(a[u][x], bb[y], acc[x][y]);
    }
  }
  if (w > 0) {
#pragma unroll
    for (int x = 0; x < TI; ++x)
#pragma unroll
      for (int y = 0; y < TJ; ++y)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[w - 1][(x * TJ + y) * 4 + e][l] = acc[x][y][e];
  }
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int x = 0; x < TI; ++x)
#pragma unroll
    for (int y = 0; y < TJ; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double v = acc[x][y][e];
        for (int ww = 0; ww < 3; ++ww) v += red[ww][(x * TJ + y) * 4 + e][l];
        const int i = (gi * TI + x) * 16 + 4 * e + kr, j = (gj * TJ + y) * 16 + cl;
        if (i < ca && j < cb) part[((size_t)i * cb + j) * gridDim.x + b] = v;
      }
}

// Y[row][j] <- sum_{i < s} Y[row][i] M[i][j] for j < sout (s, sout <= 64):
// one wave per 16-row tile, M (zero-padded to 64 x 64) in LDS; all of a
// tile's reads precede its writes (the accumulators need every k step), so
// the update is in place.
constexpr int kMfmaMaxCols = 64;

__global__ __launch_bounds__(kThreads) void k_rows_mat_mfma(int64_t n, double* __restrict__ Y, int ld,
                                                           int s, const double* __restrict__ M,
                                                           int sout) {
  // M's first s4 rows (zero-padded to 64 columns), loaded once per block;
  // the block's waves then take 16-row tiles in a grid-stride loop
  __shared__ double sM[kMfmaMaxCols * kMfmaMaxCols];
  const int s4 = (s + 3) & ~3, ntile = (sout + 15) / 16;
  for (int e = threadIdx.x; e < s4 * kMfmaMaxCols; e += kThreads) {
    const int i = e / kMfmaMaxCols, j = e % kMfmaMaxCols;
    sM[e] = (i < s && j < sout) ? M[(size_t)i * sout + j] : 0.0;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int kr = l >> 4, cl = l & 15;
  for (int64_t row0 = ((int64_t)blockIdx.x * (kThreads / 64) + w) * 16; row0 < n;
       row0 += (int64_t)gridDim.x * (kThreads / 64) * 16) {
    dmf4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = dmf4{0.0, 0.0, 0.0, 0.0};
    const int64_t arow = row0 + cl;
    for (int k0 = 0; k0 < s4; k0 += 4) {
      const int kk = k0 + kr;
      const double a = (arow < n && kk < s) ? Y[(size_t)arow * ld + kk] : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < ntile) acc[t] = mfma_f64(a, sM[kk * kMfmaMaxCols + t * 16 + cl], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < ntile)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = row0 + 4 * e + kr;
          const int j = t * 16 + cl;
          if (row < n && j < sout) Y[(size_t)row * ld + j] = acc[t][e];
        }
  }
}

// The same product with each wave's 16-row tile moved through LDS: one
// coalesced 16-byte read of the tile (row stride ld + 1 in LDS against bank
// conflicts), the same MFMA sequence on it, the result written back into the
// tile and stored with 16-byte writes (columns sout .. ld-1 keep their
// values).  Dynamic LDS: M [s4][64] and four tiles [16][ld + 1].
__global__ __launch_bounds__(kThreads) void k_rows_mat_mfma_lds(int64_t n, double* __restrict__ Y,
                                                               int ld, int s,
                                                               const double* __restrict__ M,
                                                               int sout) {
  extern __shared__ double sm[];
  const int s4 = (s + 3) & ~3, ntile = (sout + 15) / 16, st = ld + 1;
  double* sM = sm;
  for (int e = threadIdx.x; e < s4 * kMfmaMaxCols; e += kThreads) {
    const int i = e / kMfmaMaxCols, j = e % kMfmaMaxCols;
    sM[e] = (i < s && j < sout) ? M[(size_t)i * sout + j] : 0.0;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int kr = l >> 4, cl = l & 15;
  double* sT = sm + (size_t)s4 * kMfmaMaxCols + (size_t)w * 16 * st;
  const int half = ld / 2;  // 16-byte chunks per row
  // a tile of at most four 16-byte loads per lane (ld <= 32): the wave's next
  // tile is loaded into registers while this one is computed (a tile's rows
  // belong to one wave, so reading them early is safe with the in-place
  // update)
  const bool pf = 16 * half <= 4 * 64;
  const int64_t step = (int64_t)gridDim.x * (kThreads / 64) * 16;
  double2 nx[4];
  auto fetch = [&](int64_t r0) {
    const int nr = (int)min((int64_t)16, n - r0);
    const double2* src = reinterpret_cast<const double2*>(Y + (size_t)r0 * ld);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = l + 64 * i;
      if (c < nr * half) nx[i] = src[c];
    }
  };
  const int64_t first = ((int64_t)blockIdx.x * (kThreads / 64) + w) * 16;
  if (pf && first < n) fetch(first);
  for (int64_t row0 = first; row0 < n; row0 += step) {
    const int nrow = (int)min((int64_t)16, n - row0);
    if (pf) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = l + 64 * i;
        if (c < nrow * half) {
          const int r = c / half, q = 2 * (c - r * half);
          sT[r * st + q] = nx[i].x;
          sT[r * st + q + 1] = nx[i].y;
        }
      }
      if (row0 + step < n) fetch(row0 + step);
    } else {
      const double2* src = reinterpret_cast<const double2*>(Y + (size_t)row0 * ld);
      for (int c = l; c < nrow * half; c += 64) {
        const double2 v = src[c];
        const int r = c / half, q = 2 * (c - r * half);
        sT[r * st + q] = v.x;
        sT[r * st + q + 1] = v.y;
      }
    }
    wave_lds_sync();
    dmf4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = dmf4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < s4; k0 += 4) {
      const int kk = k0 + kr;
      const double a = (cl < nrow && kk < s) ? sT[cl * st + kk] : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < ntile) acc[t] = mfma_f64(a, sM[kk * kMfmaMaxCols + t * 16 + cl], acc[t]);
    }
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < ntile)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = 4 * e + kr, j = t * 16 + cl;
          if (r < nrow && j < sout) sT[r * st + j] = acc[t][e];
        }
    wave_lds_sync();
    double2* dst = reinterpret_cast<double2*>(Y + (size_t)row0 * ld);
    for (int c = l; c < nrow * half; c += 64) {
      const int r = c / half, q = 2 * (c - r * half);
      double2 v;
      v.x = sT[r * st + q];
      v.y = sT[r * st + q + 1];
      dst[c] = v;
    }
    wave_lds_sync();
  }
}

// Start block [A | G - A P] (s <= 64, r <= 256, P in LDS) and the per-block
// partial squared column norms (FP64 values before narrowing): one wave per
// 16-row tile of the block's rows, the product A P on the matrix cores in
// chunks of 4 column tiles.  Column norms: each lane sums its column over
// its rows, the four lanes of a column are combined by a fixed shuffle tree,
// the block's waves in wave order.
// MODE >= 1: each wave assembles its 16-row output tile in LDS and writes it
// with 16-byte stores (the rows of X0 are contiguous); otherwise element
// stores.  MODE 2: the wave's 16-row tile of A is read once with 16-byte
// loads into LDS (row stride lda + 1) and both uses of A read it there; when
// a tile is at most four 16-byte loads per lane (lda <= 32) the next tile's
// rows, and the sign words of its first 64 residual columns, are loaded into
// registers while the current tile is computed.  Same values in every mode.
template <typename XT, int NT, bool MASK, int MODE>
__global__ __launch_bounds__(kThreads) void k_project_mfma(int64_t n, int rpb, const double* __restrict__ A,
                                                          int lda, int s, const double* __restrict__ Gd,
                                                          int ldg, const uint64_t* __restrict__ Gmk,
                                                          int nwg, int r,
                                                          const double* __restrict__ P,
                                                          XT* __restrict__ X0, int ld,
                                                          double* __restrict__ part, double oscale) {
  extern __shared__ double sm[];
  const int r16 = (r + 15) & ~15, s4 = (s + 3) & ~3;
  constexpr bool STAGE = MODE >= 1, SA = MODE == 2;
  // P [s4][r16]; then one region for the A tiles [4 waves][16][lda + 1] (SA,
  // used inside the row loop) and the norm partials [4 waves][kMaxLd] (used
  // after it); then the output tiles [4 waves][16][ld] (STAGE)
  const int sta = lda + 1;
  const size_t nu = SA ? max((size_t)4 * kMaxLd, (size_t)4 * 16 * sta) : (size_t)4 * kMaxLd;
  double* sP = sm;
  double* sN = sm + (size_t)s4 * r16;
  double* sA = sN + (size_t)(threadIdx.x >> 6) * 16 * sta;
  XT* sO = reinterpret_cast<XT*>(sN + nu) + (size_t)(threadIdx.x >> 6) * 16 * ld;
  for (int e = threadIdx.x; e < s4 * r16; e += kThreads) {
    const int i = e / r16, j = e % r16;
    sP[e] = (i < s && j < r) ? P[(size_t)i * r + j] : 0.0;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int kr = l >> 4, cl = l & 15;
  const int64_t rb0 = (int64_t)blockIdx.x * rpb;
  const int64_t rb1 = min(n, rb0 + (int64_t)rpb);
  const int ntile = r16 / 16;
  double nrm_res[NT];   // this lane's column (16 t + cl) of the residual part (ntile <= NT)
#pragma unroll
  for (int t = 0; t < NT; ++t) nrm_res[t] = 0.0;
  double nrm_a = 0.0;   // column l of the sketch part (l < s)
  const int halfa = lda / 2;
  const bool pfa = SA && 16 * halfa <= 4 * 64;
  double2 na[4];        // the next tile's rows of A (pfa)
  uint64_t nw[4], cw[4];  // its / this tile's sign words of residual columns 0..63
  auto fetch = [&](int64_t r0) {
    const int nrow = (int)min((int64_t)16, rb1 - r0);
    const double2* src = reinterpret_cast<const double2*>(A + (size_t)r0 * lda);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = l + 64 * i;
      if (c < nrow * halfa) na[i] = src[c];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = r0 + 4 * e + kr;
      nw[e] = (MASK && row < rb1) ? Gmk[(size_t)row * nwg] : 0ull;
    }
  };
  if (pfa && rb0 + 16 * w < rb1) fetch(rb0 + 16 * w);
  for (int64_t row0 = rb0 + 16 * w; row0 < rb1; row0 += 16 * (kThreads / 64)) {
    if constexpr (SA) {
      const int nrow = (int)min((int64_t)16, rb1 - row0);
      if (pfa) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = l + 64 * i;
          if (c < nrow * halfa) {
            const int rr = c / halfa, q = 2 * (c - rr * halfa);
            sA[rr * sta + q] = na[i].x;
            sA[rr * sta + q + 1] = na[i].y;
          }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) cw[e] = nw[e];
        const int64_t next = row0 + 16 * (kThreads / 64);
        if (next < rb1) fetch(next);
      } else {
        const double2* src = reinterpret_cast<const double2*>(A + (size_t)row0 * lda);
        for (int c = l; c < nrow * halfa; c += 64) {
          const double2 v = src[c];
          const int rr = c / halfa, q = 2 * (c - rr * halfa);
          sA[rr * sta + q] = v.x;
          sA[rr * sta + q + 1] = v.y;
        }
      }
      wave_lds_sync();
    }
    // sketch columns (lane l: column l) and padding columns (lane l: s + r + l)
    if (l < s) {
      for (int q = 0; q < 16; ++q) {
        const int64_t row = row0 + q;
        if (row >= rb1) break;
        const double v = SA ? sA[q * sta + l] : A[(size_t)row * lda + l];
        if constexpr (STAGE)
          sO[q * ld + l] = XT(v * oscale);
        else
          X0[(size_t)row * ld + l] = XT(v * oscale);
        nrm_a = fma(v, v, nrm_a);
      }
    }
    if (l < ld - s - r) {
      for (int q = 0; q < 16; ++q) {
        const int64_t row = row0 + q;
        if (row >= rb1) break;
        if constexpr (STAGE)
          sO[q * ld + s + r + l] = XT(0.0);
        else
          X0[(size_t)row * ld + s + r + l] = XT(0.0);
      }
    }
    const int64_t arow = row0 + cl;
    for (int t0 = 0; t0 < ntile; t0 += 4) {
      dmf4 acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = dmf4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < s4; k0 += 4) {
        const int kk = k0 + kr;
        const double a = (arow < rb1 && kk < s)
                             ? (SA ? sA[cl * sta + kk] : A[(size_t)arow * lda + kk])
                             : 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t0 + t < ntile) acc[t] = mfma_f64(a, sP[kk * r16 + (t0 + t) * 16 + cl], acc[t]);
      }
      // sign words: tiles t0 .. t0 + 3 are columns 64 (t0 / 4) .. + 63
      uint64_t wd[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = row0 + 4 * e + kr;
        wd[e] = (pfa && t0 == 0) ? cw[e]
                                 : ((MASK && row < rb1) ? Gmk[(size_t)row * nwg + (t0 >> 2)] : 0ull);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t0 + t >= ntile) break;
        const int j = (t0 + t) * 16 + cl;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = row0 + 4 * e + kr;
          if (row < rb1 && j < r) {
            const double g = MASK ? (((wd[e] >> (j & 63)) & 1ull) ? -1.0 : 1.0)
                                  : Gd[(size_t)row * ldg + j];
            const double v = g - acc[t][e];
            if constexpr (STAGE)
              sO[(4 * e + kr) * ld + s + j] = XT(v * oscale);
            else
              X0[(size_t)row * ld + s + j] = XT(v * oscale);
            nrm_res[t0 + t] = fma(v, v, nrm_res[t0 + t]);
          }
        }
      }
    }
    if constexpr (STAGE) {
      // the tile's valid rows as 16-byte chunks (a row is a whole number of
      // chunks: ld * sizeof(XT) is a multiple of 16)
      wave_lds_sync();
      const int nrow = (int)min((int64_t)16, rb1 - row0);
      const int nck = nrow * ld * (int)sizeof(XT) / 16;
      const float4* src = reinterpret_cast<const float4*>(sO);
      float4* dst = reinterpret_cast<float4*>(X0 + (size_t)row0 * ld);
      for (int c = l; c < nck; c += 64) dst[c] = src[c];
      wave_lds_sync();
    }
  }
  // column sums: residual columns over the 4 lanes of a column, then waves
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double v = nrm_res[t];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    nrm_res[t] = v;
  }
  if constexpr (SA) __syncthreads();  // every wave is done with its A tile
  for (int c = threadIdx.x; c < 4 * kMaxLd; c += kThreads) sN[c] = 0.0;
  __syncthreads();
  if (l < s) sN[w * kMaxLd + l] = nrm_a;
  if (kr == 0)
    for (int t = 0; t < ntile; ++t)
      if (t * 16 + cl < r) sN[w * kMaxLd + s + t * 16 + cl] = nrm_res[t];
  __syncthreads();
  for (int c = threadIdx.x; c < ld; c += kThreads) {
    double v = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) v += sN[q * kMaxLd + c];
    part[(size_t)c * gridDim.x + blockIdx.x] = v;
  }
}

// Start block of the Krylov runs: columns [A | G - A P], plus per-block
// partial squared column norms (FP64 values, before any narrowing).  Rows go
// through LDS in tiles of tr: the A tile and P (when it fits) are staged,
// each thread forms 4 adjacent columns of one row of G - A P in registers,
// the finished tile [tr][ld] is assembled in LDS and written row-major, and
// thread c accumulates column c's norm in row order.
template <typename XT>
__global__ __launch_bounds__(kThreads) void k_project(int64_t n, int rpb, const double* __restrict__ A,
                                                     int lda, int s, const GSrc Gm, int r,
                                                     const double* __restrict__ P,
                                                     int p_in_lds, XT* __restrict__ X0, int ld,
                                                     int tr, double* __restrict__ part,
                                                     double oscale) {
  extern __shared__ double sm[];
  double* sa = sm;                      // [tr][s]
  double* so = sa + (size_t)tr * s;     // [tr][ld]
  double* sp = so + (size_t)tr * ld;    // [s][r] when p_in_lds
  const int lb = blockIdx.x;
  const int64_t r0 = (int64_t)lb * rpb;
  const int64_t r1 = min(n, r0 + (int64_t)rpb);
  const int t = threadIdx.x;
  if (p_in_lds)
    for (int e = t; e < s * r; e += kThreads) sp[e] = P[e];
  const double* Pp = p_in_lds ? sp : P;
  const int nq = (r + 3) / 4;
  double nacc = 0.0;
  for (int64_t rowb = r0; rowb < r1; rowb += tr) {
    const int nr = (int)min((int64_t)tr, r1 - rowb);
    __syncthreads();
    for (int e = t; e < tr * s; e += kThreads) {
      const int rr = e / s, i = e % s;
      sa[e] = (rr < nr) ? A[(size_t)(rowb + rr) * lda + i] : 0.0;
    }
    __syncthreads();
    // sketch columns and padding of the output tile
    for (int e = t; e < tr * ld; e += kThreads) {
      const int rr = e / ld, c = e % ld;
      if (c < s) so[e] = sa[rr * s + c];
      else if (c >= s + r) so[e] = 0.0;
    }
    // residual columns: 4 at a time per thread
    for (int it = t; it < tr * nq; it += kThreads) {
      const int rr = it / nq, q = it % nq;
      if (rr >= nr) continue;
      const int j0 = 4 * q;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = 0; i < s; ++i) {
        const double a = sa[rr * s + i];
        const double* pr = Pp + (size_t)i * r + j0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (j0 + u < r) acc[u] = fma(a, pr[u], acc[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j0 + u < r) so[rr * ld + s + j0 + u] = gsrc_at(Gm, rowb + rr, j0 + u) - acc[u];
    }
    __syncthreads();
    if (t < ld) {
      for (int rr = 0; rr < nr; ++rr) {
        const double v = so[rr * ld + t];
        X0[(size_t)(rowb + rr) * ld + t] = XT(v * oscale);
        nacc = fma(v, v, nacc);
      }
    }
  }
  if (t < ld) part[(size_t)t * gridDim.x + lb] = nacc;
}

// Gershgorin: per block min(a_ii - sum|a_ij|) and max(a_ii + sum|a_ij|).
__global__ __launch_bounds__(kThreads) void k_gershgorin(int64_t n, const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const double* __restrict__ va,
                                                        double* __restrict__ part) {
  __shared__ double smin[kThreads], smax[kThreads];
  const int64_t row = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  if (row < n) {
    double c = 0.0, rad = 0.0;
    for (int k = rp[row]; k < rp[row + 1]; ++k) {
      if (ci[k] == row) c += va[k];
      else rad += fabs(va[k]);
    }
    lo = c - rad;
    hi = c + rad;
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smin[0];
    part[2 * blockIdx.x + 1] = smax[0];
  }
}

hipError_t launch_gemm_tn(hipStream_t st, const Geom& g, const double* Xa, int lda, int ca,
                          const double* Xb, int ldb, int cb, double* part) {
  if (!Xb || cb > ldb) return hipErrorInvalidValue;
  return launch_gemm_tn_g(st, g, Xa, lda, ca, GSrc{Xb, ldb, nullptr, 0}, cb, part);
}

hipError_t launch_gemm_tn_g(hipStream_t st, const Geom& g, const double* Xa, int lda, int ca,
                            const GSrc& Xb, int cb, double* part) {
  if (g.n < 1 || g.nblk < 1 || !Xa || !part || ca < 1 || cb < 1 || ca > lda ||
      (int64_t)g.nblk * g.rpb < g.n || (!Xb.dense) == (!Xb.mask) ||
      (Xb.dense && cb > Xb.ld) || (Xb.mask && Xb.nw != (cb + 63) / 64))
    return hipErrorInvalidValue;
  // 2 x 2 tiles of 16 x 16 per wave on the matrix cores; 2 x 4 for a wider
  // right operand that is not the left one (each row of Xa then read once per
  // 64 columns of Xb instead of per 32)
  const int ngi = (ca + 31) / 32;
  if (cb > 32 && Xa != Xb.dense) {
    const int ngj = (cb + 63) / 64;
    auto fn = Xb.mask ? k_gemm_tn_mfma<2, 4, true> : k_gemm_tn_mfma<2, 4, false>;
    hipLaunchKernelGGL(fn, dim3(g.nblk, ngi * ngj), dim3(kThreads), 0, st, g.n, g.rpb, Xa, lda, ca,
                       Xb.dense, Xb.ld, Xb.mask, Xb.nw, cb, ngj, part);
    return hipGetLastError();
  }
  const int ngj = (cb + 31) / 32;
  auto fn = Xb.mask ? k_gemm_tn_mfma<2, 2, true> : k_gemm_tn_mfma<2, 2, false>;
  hipLaunchKernelGGL(fn, dim3(g.nblk, ngi * ngj), dim3(kThreads), 0, st, g.n, g.rpb, Xa, lda, ca,
                     Xb.dense, Xb.ld, Xb.mask, Xb.nw, cb, ngj, part);
  return hipGetLastError();
}

hipError_t launch_chol_inv(hipStream_t st, int s, const double* G, double* work, double* Rinv,
                           int* flag) {
  if (s < 1 || s > 256 || !G || !work || !Rinv || !flag) return hipErrorInvalidValue;
  if (s <= kCholLdsMax)
    hipLaunchKernelGGL(k_chol_inv_lds, dim3(1), dim3(kThreads), (size_t)2 * s * s * sizeof(double),
                       st, s, G, work, Rinv, flag);
  else
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kThreads), 0, st, s, G, work, Rinv, flag);
  return hipGetLastError();
}

// Y <- Y M on the matrix cores (s, sout <= 64): through LDS tiles when they
// fit, else straight from global memory.
static hipError_t rows_mat_mfma(hipStream_t st, int64_t n, double* Y, int ld, int s,
                                const double* M, int sout) {
  const int64_t tiles = (n + 15) / 16;
  const int64_t nb = std::min<int64_t>((tiles + 3) / 4, 2 * kMaxBlocks);
  const size_t lds = ((size_t)((s + 3) & ~3) * kMfmaMaxCols + (size_t)4 * 16 * (ld + 1)) *
                     sizeof(double);
  if (ld % 2 == 0 && lds <= 64 * 1024 && reinterpret_cast<uintptr_t>(Y) % 16 == 0)
    hipLaunchKernelGGL(k_rows_mat_mfma_lds, dim3((unsigned)nb), dim3(kThreads), lds, st, n, Y, ld,
                       s, M, sout);
  else
    hipLaunchKernelGGL(k_rows_mat_mfma, dim3((unsigned)nb), dim3(kThreads), 0, st, n, Y, ld, s, M,
                       sout);
  return hipGetLastError();
}

hipError_t launch_trsm_rows(hipStream_t st, int64_t n, double* Y, int ld, int s, const double* Rinv) {
  if (n < 1 || s < 1 || s > 256 || ld < s || !Y || !Rinv) return hipErrorInvalidValue;
  if (s <= kMfmaMaxCols) return rows_mat_mfma(st, n, Y, ld, s, Rinv, s);
  const size_t lds = (size_t)(16 * s + 16 * s) * sizeof(double);
  hipLaunchKernelGGL(k_rows_mat<true>, dim3((unsigned)((n + 15) / 16)), dim3(kThreads), lds, st, n, Y,
                     ld, s, Rinv, s);
  return hipGetLastError();
}

hipError_t launch_rows_mat(hipStream_t st, int64_t n, double* Y, int ld, int s, const double* M,
                           int sout) {
  if (n < 1 || s < 1 || s > 256 || sout < 1 || sout > s || ld < s || !Y || !M)
    return hipErrorInvalidValue;
  if (s <= kMfmaMaxCols) {
    return rows_mat_mfma(st, n, Y, ld, s, M, sout);
  }
  const size_t lds = (size_t)(16 * s + 16 * s) * sizeof(double);
  hipLaunchKernelGGL(k_rows_mat<false>, dim3((unsigned)((n + 15) / 16)), dim3(kThreads), lds, st, n, Y,
                     ld, s, M, sout);
  return hipGetLastError();
}

hipError_t launch_subspace_eig(hipStream_t st, int q, int k, const double* G, double* U, int* flag) {
  if (q < 1 || q > kEigMax || k < 1 || k > q || !G || !U || !flag) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_subspace_eig, dim3(1), dim3(kThreads), 0, st, q, k, G, U, flag);
  return hipGetLastError();
}

hipError_t launch_project(hipStream_t st, const Geom& g, const double* A, int lda, int s,
                          const GSrc& Gm, int r, const double* P, void* X0, double* part,
                          double oscale) {
  if (g.n < 1 || g.nblk < 1 || (int64_t)g.nblk * g.rpb < g.n || !X0 || !part || r < 1 ||
      s < 0 || s + r > g.ld || g.ld > kThreads || (s > 0 && (!A || !P || lda < s)) ||
      (!Gm.dense) == (!Gm.mask) || (Gm.dense && Gm.ld < r) ||
      (Gm.mask && Gm.nw != (r + 63) / 64) || !(oscale > 0.0))
    return hipErrorInvalidValue;
  {
    // matrix cores when P (and the norm partials) fit the block's LDS
    const size_t r16 = (size_t)((r + 15) & ~15), s4 = (size_t)((s + 3) & ~3);
    const size_t lds_m = (s4 * r16 + 4 * kMaxLd) * sizeof(double);
    // with the output tiles staged when they fit
    const size_t lds_st = lds_m + (size_t)4 * 16 * g.ld * g.xbytes;
    const bool stage = lds_st <= 64 * 1024 && (g.ld * g.xbytes) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(X0) % 16 == 0;
    const size_t lds_sa =
        ((size_t)s4 * r16 + std::max((size_t)4 * kMaxLd, (size_t)4 * 16 * (lda + 1))) *
            sizeof(double) +
        (size_t)4 * 16 * g.ld * g.xbytes;
    const bool stage_a = stage && s > 0 && lds_sa <= 64 * 1024 && lda % 2 == 0 &&
                         reinterpret_cast<uintptr_t>(A) % 16 == 0;
    const int mode = stage_a ? 2 : (stage ? 1 : 0);
    if (s <= kMfmaMaxCols && r <= 256 && lds_m <= 64 * 1024) {
      // residual column tiles held per lane: 4, 8 or 16
      const int nt = (int)(r16 / 16);
      auto go = [&](auto xt_tag, auto nt_tag) {
        using XTT = decltype(xt_tag);
        constexpr int NT = decltype(nt_tag)::value;
        auto pick = [&](auto mask_tag) {
          constexpr bool MK = decltype(mask_tag)::value;
          return mode == 2 ? k_project_mfma<XTT, NT, MK, 2>
                           : (mode == 1 ? k_project_mfma<XTT, NT, MK, 1>
                                        : k_project_mfma<XTT, NT, MK, 0>);
        };
        auto fn = Gm.mask ? pick(std::true_type{}) : pick(std::false_type{});
        const size_t lds = mode == 2 ? lds_sa : (mode == 1 ? lds_st : lds_m);
        hipLaunchKernelGGL(fn, dim3(g.nblk), dim3(kThreads), lds, st, g.n, g.rpb, A, lda, s,
                           Gm.dense, Gm.ld, Gm.mask, Gm.nw, r, P, static_cast<XTT*>(X0), g.ld,
                           part, oscale);
      };
      auto by_nt = [&](auto xt_tag) {
        if (nt <= 4)
          go(xt_tag, std::integral_constant<int, 4>{});
        else if (nt <= 8)
          go(xt_tag, std::integral_constant<int, 8>{});
        else
          go(xt_tag, std::integral_constant<int, 16>{});
      };
      if (g.xbytes == 8)
        by_nt(double{});
      else if (g.xbytes == 4)
        by_nt(float{});
      else
        by_nt(_Float16{});
      return hipGetLastError();
    }
  }
  // largest row tile (32, 16 or 8) whose staging fits 64 KB, P staged too when it fits
  const size_t budget = 64 * 1024;
  int tr = 32;
  while (tr > 8 && (size_t)tr * (s + g.ld) * sizeof(double) > budget) tr /= 2;
  size_t lds = (size_t)tr * (s + g.ld) * sizeof(double);
  if (lds > budget) return hipErrorInvalidValue;
  int p_in_lds = 0;
  if (s > 0 && lds + (size_t)s * r * sizeof(double) <= budget) {
    p_in_lds = 1;
    lds += (size_t)s * r * sizeof(double);
  }
  if (g.xbytes == 8)
    hipLaunchKernelGGL(k_project<double>, dim3(g.nblk), dim3(kThreads), lds, st, g.n, g.rpb, A, lda,
                       s, Gm, r, P, p_in_lds, static_cast<double*>(X0), g.ld, tr, part, oscale);
  else if (g.xbytes == 4)
    hipLaunchKernelGGL(k_project<float>, dim3(g.nblk), dim3(kThreads), lds, st, g.n, g.rpb, A, lda,
                       s, Gm, r, P, p_in_lds, static_cast<float*>(X0), g.ld, tr, part, oscale);
  else
    hipLaunchKernelGGL(k_project<_Float16>, dim3(g.nblk), dim3(kThreads), lds, st, g.n, g.rpb, A,
                       lda, s, Gm, r, P, p_in_lds, static_cast<_Float16*>(X0), g.ld, tr, part,
                       oscale);
  return hipGetLastError();
}

hipError_t launch_gershgorin(hipStream_t st, int64_t n, const int* rp, const int* ci,
                             const double* va, double* part, int* nparts) {
  if (n < 1 || !rp || !ci || !va || !part || !nparts) return hipErrorInvalidValue;
  const int nb = (int)((n + kThreads - 1) / kThreads);
  *nparts = nb;
  hipLaunchKernelGGL(k_gershgorin, dim3(nb), dim3(kThreads), 0, st, n, rp, ci, va, part);
  return hipGetLastError();
}

}  // namespace ld
