// log(H) e1 for the small Hessenberg matrix of an Arnoldi/IOP run (Alg 1),
// shared by the GPU kernel (one workgroup per run) and a host unit test.
//
// Method: inverse scaling and squaring.  Take square roots A <- A^{1/2}
// (Denman-Beavers iteration in product form: M0 = Y0 = A,
// Y <- Y (I + M^{-1}) / 2, M <- (I + (M + M^{-1}) / 2) / 2, so Y -> A^{1/2},
// M -> I) until ||A - I||_1 <= 1/4, then
//   log(A) = 2^s log(I + X),  X = A^{1/2^s} - I,
//   log(I + X) = int_0^1 X (I + t X)^{-1} dt ~ sum_j w_j (I + x_j X)^{-1} X,
// the Gauss-Legendre rule in t being the [k/k] Pade approximant of log(1+x)
// (Higham, "Evaluating Pade approximants of the matrix logarithm", 2001).
// Only log(A) e1 is needed: sum_j w_j (I + x_j X)^{-1} (X e1), one linear
// solve per node.  Each square root multiplies the eigenvalues' logarithms
// by 1/2, so the principal branch is kept when the spectrum avoids the
// closed negative real axis (true for the projections of an SPD operator).
//
// Parallel structure: a team of nt threads sharing memory (a GPU workgroup,
// or one host thread); all matrices are n x n row-major (leading dimension
// n) in memory visible to the team.  Control flow is uniform across the team.
#pragma once

#include <math.h>

#ifndef LD_HD
#if defined(__HIPCC__)
#define LD_HD __host__ __device__
#else
#define LD_HD
#endif
#endif

namespace ld {

constexpr int kLogNodes = 10;  // Gauss-Legendre nodes of the Pade step

struct HostTeam {
  int tid() const { return 0; }
  int nt() const { return 1; }
  void sync() const {}
};

#if defined(__HIPCC__)
struct BlockTeam {
  __device__ int tid() const { return (int)threadIdx.x; }
  __device__ int nt() const { return (int)blockDim.x; }
  __device__ void sync() const { __syncthreads(); }
};
#endif

// Shared scratch of a team: at least nt doubles + nt ints + 4 of each.
struct TeamScratch {
  double* d;
  int* i;
};

template <class T>
LD_HD inline void team_set_identity(const T& tm, int n, double* A, double diag) {
  for (int e = tm.tid(); e < n * n; e += tm.nt()) A[e] = (e / n == e % n) ? diag : 0.0;
}

template <class T>
LD_HD inline void team_copy(const T& tm, int count, const double* src, double* dst) {
  for (int e = tm.tid(); e < count; e += tm.nt()) dst[e] = src[e];
}

// C = alpha * A B (C distinct from A and B)
template <class T>
LD_HD inline void team_matmul(const T& tm, int n, const double* A, const double* B, double* C,
                              double alpha) {
  for (int e = tm.tid(); e < n * n; e += tm.nt()) {
    const int i = e / n, j = e % n;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc = fma(A[i * n + k], B[k * n + j], acc);
    C[e] = alpha * acc;
  }
}

// ||A - I||_1 (max column sum); every thread gets the result.
template <class T>
LD_HD inline double team_norm1_minus_identity(const T& tm, int n, const double* A, TeamScratch sc) {
  double best = 0.0;
  for (int j = tm.tid(); j < n; j += tm.nt()) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += fabs(A[i * n + j] - (i == j ? 1.0 : 0.0));
    best = (s > best || s != s) ? s : best;
  }
  sc.d[tm.tid()] = best;
  tm.sync();
  if (tm.tid() == 0) {
    double m = 0.0;
    for (int q = 0; q < tm.nt(); ++q) m = (sc.d[q] > m || sc.d[q] != sc.d[q]) ? sc.d[q] : m;
    sc.d[tm.nt()] = m;
  }
  tm.sync();
  const double r = sc.d[tm.nt()];
  tm.sync();
  return r;
}

// Gauss-Jordan elimination with partial pivoting: reduces A (destroyed) to
// the identity while applying the same row operations to R (n x nrhs), so R
// becomes A^{-1} R.  fac: n doubles of team-visible scratch.  Returns false
// (on every thread) when a pivot is zero or not finite.
template <class T>
LD_HD inline bool team_gauss_jordan(const T& tm, int n, double* A, double* R, int nrhs, double* fac,
                                    TeamScratch sc) {
  for (int k = 0; k < n; ++k) {
    // pivot: largest |A[i][k]|, i >= k (smallest index on ties)
    double bv = -1.0;
    int bi = k;
    for (int i = k + tm.tid(); i < n; i += tm.nt()) {
      const double v = fabs(A[i * n + k]);
      if (v > bv) { bv = v; bi = i; }
    }
    sc.d[tm.tid()] = bv;
    sc.i[tm.tid()] = bi;
    tm.sync();
    if (tm.tid() == 0) {
      double v = -1.0;
      int idx = k;
      for (int q = 0; q < tm.nt(); ++q)
        if (sc.d[q] > v || (sc.d[q] == v && sc.i[q] < idx)) { v = sc.d[q]; idx = sc.i[q]; }
      sc.i[tm.nt()] = idx;
      sc.d[tm.nt()] = A[idx * n + k];
    }
    tm.sync();
    const int piv = sc.i[tm.nt()];
    const double pv = sc.d[tm.nt()];
    tm.sync();
    if (!(fabs(pv) > 0.0) || !isfinite(pv)) return false;
    if (piv != k) {
      for (int j = tm.tid(); j < n; j += tm.nt()) {
        const double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t;
      }
      for (int j = tm.tid(); j < nrhs; j += tm.nt()) {
        const double t = R[k * nrhs + j]; R[k * nrhs + j] = R[piv * nrhs + j]; R[piv * nrhs + j] = t;
      }
      tm.sync();
    }
    const double inv = 1.0 / pv;
    for (int j = tm.tid(); j < n; j += tm.nt()) A[k * n + j] *= inv;
    for (int j = tm.tid(); j < nrhs; j += tm.nt()) R[k * nrhs + j] *= inv;
    for (int i = tm.tid(); i < n; i += tm.nt()) fac[i] = (i == k) ? 0.0 : A[i * n + k];
    tm.sync();
    for (int e = tm.tid(); e < n * n; e += tm.nt()) {
      const int i = e / n, j = e % n;
      if (i != k) A[e] = fma(-fac[i], A[k * n + j], A[e]);
    }
    for (int e = tm.tid(); e < n * nrhs; e += tm.nt()) {
      const int i = e / nrhs, j = e % nrhs;
      if (i != k) R[e] = fma(-fac[i], R[k * nrhs + j], R[e]);
    }
    tm.sync();
  }
  return true;
}

// Workspace doubles needed by team_hess_log_e1 for an n x n matrix.
LD_HD inline int hess_log_workspace(int n) { return 6 * n * n + 3 * n; }

// ell = log(H) e1 for the n x n matrix H (row i at H + i*hld).  nodes/weights:
// kLogNodes Gauss-Legendre points on [0, 1].  Returns 0 on success, 1 when a
// linear system was singular, 2 when the square roots did not converge.
template <class T>
LD_HD inline int team_hess_log_e1(const T& tm, int n, const double* H, int hld, double* ell,
                                  double* ws, TeamScratch sc, const double* nodes,
                                  const double* weights) {
  double* A = ws;              // current matrix
  double* M = ws + n * n;      // Denman-Beavers M
  double* Y = ws + 2 * n * n;  // Denman-Beavers Y (square root)
  double* Z = ws + 3 * n * n;  // inverse / scratch
  double* W = ws + 4 * n * n;  // scratch
  double* V = ws + 5 * n * n;  // scratch
  double* fac = ws + 6 * n * n;
  double* b = fac + n;
  double* z = b + n;
  for (int e = tm.tid(); e < n * n; e += tm.nt()) A[e] = H[(e / n) * hld + e % n];
  tm.sync();
  int s = 0;
  for (;;) {
    const double nrm = team_norm1_minus_identity(tm, n, A, sc);
    if (!(nrm == nrm)) return 2;
    if (nrm <= 0.25 || s >= 60) break;
    // A <- A^{1/2}
    team_copy(tm, n * n, A, M);
    team_copy(tm, n * n, A, Y);
    tm.sync();
    bool conv = false;
    for (int it = 0; it < 100; ++it) {
      team_copy(tm, n * n, M, W);
      team_set_identity(tm, n, Z, 1.0);
      tm.sync();
      if (!team_gauss_jordan(tm, n, W, Z, n, fac, sc)) return 1;  // Z = M^{-1}
      // V = I + M^{-1};  Y <- Y V / 2;  M <- (I + (M + M^{-1}) / 2) / 2
      for (int e = tm.tid(); e < n * n; e += tm.nt()) V[e] = Z[e] + ((e / n == e % n) ? 1.0 : 0.0);
      tm.sync();
      team_matmul(tm, n, Y, V, W, 0.5);
      for (int e = tm.tid(); e < n * n; e += tm.nt())
        M[e] = 0.25 * (M[e] + Z[e]) + ((e / n == e % n) ? 0.5 : 0.0);
      tm.sync();
      team_copy(tm, n * n, W, Y);
      tm.sync();
      const double d = team_norm1_minus_identity(tm, n, M, sc);
      if (!(d == d)) return 2;
      if (d <= 1e-15 * n) {
        conv = true;
        break;
      }
    }
    if (!conv) return 2;
    team_copy(tm, n * n, Y, A);
    tm.sync();
    ++s;
  }
  // X = A - I, b = X e1
  for (int e = tm.tid(); e < n * n; e += tm.nt()) A[e] -= (e / n == e % n) ? 1.0 : 0.0;
  tm.sync();
  for (int i = tm.tid(); i < n; i += tm.nt()) {
    b[i] = A[i * n];
    ell[i] = 0.0;
  }
  tm.sync();
  for (int q = 0; q < kLogNodes; ++q) {
    for (int e = tm.tid(); e < n * n; e += tm.nt())
      W[e] = nodes[q] * A[e] + ((e / n == e % n) ? 1.0 : 0.0);
    for (int i = tm.tid(); i < n; i += tm.nt()) z[i] = b[i];
    tm.sync();
    if (!team_gauss_jordan(tm, n, W, z, 1, fac, sc)) return 1;
    for (int i = tm.tid(); i < n; i += tm.nt()) ell[i] = fma(weights[q], z[i], ell[i]);
    tm.sync();
  }
  const double scale = ldexp(1.0, s);
  for (int i = tm.tid(); i < n; i += tm.nt()) ell[i] *= scale;
  tm.sync();
  return 0;
}

}  // namespace ld
